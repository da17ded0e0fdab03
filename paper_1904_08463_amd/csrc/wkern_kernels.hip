// HIP kernels for w-projection kernel generation on gfx950 (MI355X).
//
// Pipeline of one generate call (Lucas, Skipper & Scaife 2019, Algorithm 2):
//   k_screen_*     image-domain kernel s[i, p] = tau_i exp(+j 2 pi w_p phi_i)
//                  (section 2.5, eq. wproj_G, times the IAA-kernel), phase
//                  reduced in FP64;
//   k_contract_*   order-0 Hankel transform as K = M s on the matrix cores
//                  (section 4.3, eq. ht; the HT matrix M is built once per
//                  plan by k_hankel_matrix);
//   k_spline       spline coefficients of each radial line (section 4.3.2);
//   k_resample     oversampled 2D kernels over the circular support
//                  (section 4.4, Algorithm 2), in wkern_resample.hip.
#include <cmath>
#include <type_traits>

#include "wkern_internal.h"
#include "wkern_radial.h"

namespace wkern {

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f(uint16_t h) {
  return __uint_as_float((uint32_t)h << 16);
}

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) {
  return __builtin_bit_cast(bf16x8, v);
}

// The six split-BF16 products of one 16-node step, interleaved over the
// output blocks (rb, cb) so that consecutive MFMAs are independent: the five
// small products (02, 11, 20, 01, 10) accumulate into lo, the 00 product
// into hi (block b = rb * CBW + cb).
template <int RBW, int CBW>
__device__ __forceinline__ void mfma_split6(const bf16x8 (&aq)[RBW][3], const bf16x8 (&bq)[CBW][3],
                                            f32x16 (&lo)[RBW * CBW], f32x16 (&hi)[RBW * CBW]) {
#pragma unroll
  for (int term = 0; term < 6; ++term) {
#pragma unroll
    for (int rb = 0; rb < RBW; ++rb) {
#pragma unroll
      for (int cb = 0; cb < CBW; ++cb) {
        const int b = rb * CBW + cb;
        switch (term) {
          case 0: lo[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aq[rb][0], bq[cb][2], lo[b], 0, 0, 0); break;
          case 1: lo[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aq[rb][1], bq[cb][1], lo[b], 0, 0, 0); break;
          case 2: lo[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aq[rb][2], bq[cb][0], lo[b], 0, 0, 0); break;
          case 3: lo[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aq[rb][0], bq[cb][1], lo[b], 0, 0, 0); break;
          case 4: lo[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aq[rb][1], bq[cb][0], lo[b], 0, 0, 0); break;
          default: hi[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aq[rb][0], bq[cb][0], hi[b], 0, 0, 0); break;
        }
      }
    }
  }
}

// End of a sub-chunk: the FP32 sums of the 00 product (hi) and of the small
// products (lo) go into FP64 running sums, and start again from zero.
template <int NB>
__device__ __forceinline__ void flush_fp64(double (&accd)[NB][16], f32x16 (&hi)[NB],
                                           f32x16 (&lo)[NB]) {
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      accd[b][r] += (double)hi[b][r] + (double)lo[b][r];
      hi[b][r] = 0.f;
      lo[b][r] = 0.f;
    }
}

// End of a sub-chunk when the small products are left in their FP32
// accumulator: only the 00 product's FP32 sum goes into the FP64 running sum.
template <int NB>
__device__ __forceinline__ void flush_hi_fp64(double (&accd)[NB][16], f32x16 (&hi)[NB]) {
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      accd[b][r] += (double)hi[b][r];
      hi[b][r] = 0.f;
    }
}

// --------------------------------------------------------------------------
// Discrete HT matrix (section 4.3): M[k, i] = 2 pi J0(2 pi rho_k r_i) r_i dr,
// midpoint nodes r_i = (i + 1/2) dr, rho_k = k drho.  FP64 with the device
// j0; stored as FP32 and as three BF16 terms split from the FP64 value,
// grouped by 8 radial nodes: Msplit[k][i/8][term][i%8] (when Msplit is not
// null).
// --------------------------------------------------------------------------
__global__ void k_hankel_matrix(int rowsPad, int NrPad, int Nr, int nrhoMax, double dr,
                                double drho, float* __restrict__ M32,
                                uint16_t* __restrict__ Msplit, uint16_t* __restrict__ MsplitG) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (i >= NrPad || k >= rowsPad) return;
  double m = 0.0;
  if (i < Nr && k < nrhoMax) {
    const double r = (i + 0.5) * dr;
    const double rho = k * drho;
    m = kTwoPi * j0(kTwoPi * rho * r) * r * dr;
  }
  M32[(size_t)k * NrPad + i] = (float)m;
  if (!Msplit && !MsplitG) return;  // terms only for the variants that read them
  const uint16_t t0 = bf16_rne((float)m);
  double rem = m - (double)bf16_to_f(t0);
  const uint16_t t1 = bf16_rne((float)rem);
  rem -= (double)bf16_to_f(t1);
  const uint16_t t2 = bf16_rne((float)rem);
  if (Msplit) {
    const size_t base = ((size_t)k * (NrPad / 8) + (i >> 3)) * 24 + (i & 7);
    Msplit[base] = t0;
    Msplit[base + 8] = t1;
    Msplit[base + 16] = t2;
  }
  if (MsplitG) {
    const size_t gterm = (size_t)rowsPad * 8;  // one term of one node group
    const size_t base = (size_t)(i >> 3) * 3 * gterm + (size_t)k * 8 + (i & 7);
    MsplitG[base] = t0;
    MsplitG[base + gterm] = t1;
    MsplitG[base + 2 * gterm] = t2;
  }
}

// --------------------------------------------------------------------------
// Screen (section 2.5 eq. wproj_G times the IAA-kernel, Algorithm 2):
// s = tau exp(+j 2 pi w phi).  t = w phi is reduced modulo 1 in FP64; the
// FP32 sincospi of the reduced phase is corrected to first order with the
// FP64 remainder, so the value is accurate well beyond FP32 rounding of t.
// --------------------------------------------------------------------------
__device__ __forceinline__ float2 screen_value(double wv, double ph, float tau) {
  double t = wv * ph;
  t -= rint(t);
  const float th = (float)t;
  const float dl = (float)((t - (double)th) * kTwoPi);
  float sn, cs;
  sincospif(2.0f * th, &sn, &cs);
  const float c2 = cs - dl * sn;
  const float s2 = sn + dl * cs;
  return make_float2(tau * c2, tau * s2);
}

// FP32 screen: B32[2j + c][i], sorted plane j, c = 0 (re) / 1 (im).  A
// thread computes four consecutive nodes and writes each row's four values
// with one 16-byte store (NrPad is a multiple of 256).  A workgroup walks
// planes j0 + blockIdx.y, + gridDim.y, ...: the nodes' phi and taper are
// loaded once, and the next plane's w is loaded while the current one is
// computed.
__global__ __launch_bounds__(256) void k_screen_f32(int j0, int j1, int Nr, int NrPad,
                                                    const int32_t* __restrict__ perm,
                                                    const double* __restrict__ phi,
                                                    const float* __restrict__ taper,
                                                    const double* __restrict__ w,
                                                    float* __restrict__ B32) {
  const int i0 = 4 * (blockIdx.x * blockDim.x + threadIdx.x);
  int j = j0 + (int)blockIdx.y;
  if (i0 >= NrPad || j >= j1) return;
  double ph[4];
  float ta[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    ph[u] = i0 + u < Nr ? phi[i0 + u] : 0.0;
    ta[u] = i0 + u < Nr ? taper[i0 + u] : 0.f;
  }
  double wv = w[perm[j]];
  while (j < j1) {
    const int jn = j + (int)gridDim.y;
    const double wn = jn < j1 ? w[perm[jn]] : 0.0;
    float4 re = make_float4(0.f, 0.f, 0.f, 0.f), im = re;
    float2 v;
    if (i0 < Nr) { v = screen_value(wv, ph[0], ta[0]); re.x = v.x; im.x = v.y; }
    if (i0 + 1 < Nr) { v = screen_value(wv, ph[1], ta[1]); re.y = v.x; im.y = v.y; }
    if (i0 + 2 < Nr) { v = screen_value(wv, ph[2], ta[2]); re.z = v.x; im.z = v.y; }
    if (i0 + 3 < Nr) { v = screen_value(wv, ph[3], ta[3]); re.w = v.x; im.w = v.y; }
    *(float4*)(B32 + (size_t)(2 * j) * NrPad + i0) = re;
    *(float4*)(B32 + (size_t)(2 * j + 1) * NrPad + i0) = im;
    j = jn;
    wv = wn;
  }
}

// FP32 screen, node-group-major: B32[i / 16][c][i % 16] with c = 2 j + re/im
// (colsPad columns a group).  A workgroup takes one group of 16 nodes and
// 64 kScreenPlaneRun planes; thread 4 jj + q holds nodes 4 q .. 4 q + 3 of
// the group (their phi and taper loaded once) and walks planes jj, jj + 64,
// ..., loading the next plane's w while it computes the current one.  For
// each plane it writes the four values to the plane's re row and im row
// with one 16-byte store each: the four threads of a plane fill its 128
// contiguous bytes of the group, so a store instruction covers 16 planes'
// halves of 128-byte lines and the next instruction the other halves.
constexpr int kScreenPlaneRun = 8;
__global__ __launch_bounds__(256) void k_screen_f32_groups(int j0, int j1, int Nr, int colsPad,
                                                           const int32_t* __restrict__ perm,
                                                           const double* __restrict__ phi,
                                                           const float* __restrict__ taper,
                                                           const double* __restrict__ w,
                                                           float* __restrict__ B32) {
  const int q = (int)(threadIdx.x & 3);
  const int g = (int)blockIdx.y;
  const int i0 = 16 * g + 4 * q;
  int j = j0 + 64 * kScreenPlaneRun * (int)blockIdx.x + (int)(threadIdx.x >> 2);
  if (j >= j1) return;
  double ph[4];
  float ta[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    ph[u] = i0 + u < Nr ? phi[i0 + u] : 0.0;
    ta[u] = i0 + u < Nr ? taper[i0 + u] : 0.f;
  }
  const int jEnd = min(j1, j + 64 * kScreenPlaneRun);
  double wv = w[perm[j]];
  float* row = B32 + ((size_t)g * colsPad + 2 * j) * 16 + 4 * q;
  while (j < jEnd) {
    const int jn = j + 64;
    const double wn = jn < jEnd ? w[perm[jn]] : 0.0;
    float4 re = make_float4(0.f, 0.f, 0.f, 0.f), im = re;
    float2 v;
    if (i0 < Nr) { v = screen_value(wv, ph[0], ta[0]); re.x = v.x; im.x = v.y; }
    if (i0 + 1 < Nr) { v = screen_value(wv, ph[1], ta[1]); re.y = v.x; im.y = v.y; }
    if (i0 + 2 < Nr) { v = screen_value(wv, ph[2], ta[2]); re.z = v.x; im.z = v.y; }
    if (i0 + 3 < Nr) { v = screen_value(wv, ph[3], ta[3]); re.w = v.x; im.w = v.y; }
    *(float4*)row = re;
    *(float4*)(row + 16) = im;
    row += 64 * 2 * 16;
    j = jn;
    wv = wn;
  }
}

// Split-BF16 screen: Bsplit[col][i/8][term][i%8]; one thread per 8 nodes.
__global__ void k_screen_bf16(int j0, int j1, int Nr, int NrPad,
                              const int32_t* __restrict__ perm, const double* __restrict__ phi,
                              const float* __restrict__ taper, const double* __restrict__ w,
                              uint16_t* __restrict__ Bsplit) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;  // group of 8 nodes
  const int ng = NrPad / 8;
  if (g >= ng) return;
  for (int j = j0 + blockIdx.y; j < j1; j += gridDim.y) {
    const double wv = w[perm[j]];
    uint16_t re[3][8], im[3][8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int i = g * 8 + e;
      float2 v = make_float2(0.f, 0.f);
      if (i < Nr) v = screen_value(wv, phi[i], taper[i]);
      float x = v.x;
      uint16_t a0 = bf16_rne(x);
      x -= bf16_to_f(a0);
      uint16_t a1 = bf16_rne(x);
      x -= bf16_to_f(a1);
      re[0][e] = a0;
      re[1][e] = a1;
      re[2][e] = bf16_rne(x);
      float y = v.y;
      uint16_t b0 = bf16_rne(y);
      y -= bf16_to_f(b0);
      uint16_t b1 = bf16_rne(y);
      y -= bf16_to_f(b1);
      im[0][e] = b0;
      im[1][e] = b1;
      im[2][e] = bf16_rne(y);
    }
    uint4* dre = (uint4*)(Bsplit + ((size_t)(2 * j) * ng + g) * 24);
    uint4* dim = (uint4*)(Bsplit + ((size_t)(2 * j + 1) * ng + g) * 24);
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      uint4 a, b;
      a.x = re[t][0] | ((uint32_t)re[t][1] << 16);
      a.y = re[t][2] | ((uint32_t)re[t][3] << 16);
      a.z = re[t][4] | ((uint32_t)re[t][5] << 16);
      a.w = re[t][6] | ((uint32_t)re[t][7] << 16);
      b.x = im[t][0] | ((uint32_t)im[t][1] << 16);
      b.y = im[t][2] | ((uint32_t)im[t][3] << 16);
      b.z = im[t][4] | ((uint32_t)im[t][5] << 16);
      b.w = im[t][6] | ((uint32_t)im[t][7] << 16);
      dre[t] = a;
      dim[t] = b;
    }
  }
}

// --------------------------------------------------------------------------
// Hankel contraction K[k, c] = sum_i M[k, i] B[c, i] over one K-chunk of a
// tile.  One wave per tile of 32 rows x 32*CB columns; 32x32 MFMA output
// blocks (lane l holds column l%32, rows 8*(r/4) + 4*(l/32) + r%4 of its
// 16 accumulators).  The radial index is permuted identically for A and B
// inside each K-step, which leaves the sum unchanged.  Every kSubChunk nodes
// the FP32 matrix-core sums are added to FP64 running sums.
// --------------------------------------------------------------------------
template <int CB>
__device__ __forceinline__ void store_tile(const Tile& t, const double (*accd)[16], int P,
                                           int lineTotal, const int32_t* __restrict__ nrhoSorted,
                                           const int32_t* __restrict__ lineOffSorted,
                                           double* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int hb = lane >> 5;
  const int rr = lane & 31;
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const int col = t.col0 + 32 * cb + rr;
    const int j = col >> 1;
    const int comp = col & 1;
    if (j >= P || j >= t.pad[0]) continue;  // pad[0]: end of the tile's chunk
    const int nr = nrhoSorted[j];
    double* dst = part + ((size_t)t.kc * lineTotal + lineOffSorted[j]) * 2 + comp;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = t.row0 + 8 * (r >> 2) + 4 * hb + (r & 3);
      if (row < nr) dst[(size_t)row * 2] = accd[cb][r];
    }
  }
}

template <int CB>
__global__ __launch_bounds__(64) void k_contract_f32(
    const Tile* __restrict__ tiles, int NrPad, int kchunk, int P, int lineTotal,
    const float* __restrict__ M32, const float* __restrict__ B32,
    const int32_t* __restrict__ nrhoSorted, const int32_t* __restrict__ lineOffSorted,
    double* __restrict__ part) {
  const Tile t = tiles[blockIdx.x];
  if (t.row0 < 0) return;
  const int lane = threadIdx.x;
  const int hb = lane >> 5;
  const int rr = lane & 31;
  const float* arow = M32 + (size_t)(t.row0 + rr) * NrPad + 4 * hb;
  const float* bcol[CB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) bcol[cb] = B32 + (size_t)(t.col0 + 32 * cb + rr) * NrPad + 4 * hb;
  double accd[CB][16];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb)
#pragma unroll
    for (int r = 0; r < 16; ++r) accd[cb][r] = 0.0;

  for (int ks = t.k0; ks < t.k0 + kchunk; ks += kSubChunk) {
    f32x16 acc[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[cb][r] = 0.f;
#pragma unroll 4
    for (int k0 = ks; k0 < ks + kSubChunk; k0 += 8) {
      const float4 a4 = *(const float4*)(arow + k0);
      float4 b4[CB];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) b4[cb] = *(const float4*)(bcol[cb] + k0);
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.x, b4[cb].x, acc[cb], 0, 0, 0);
        acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.y, b4[cb].y, acc[cb], 0, 0, 0);
        acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.z, b4[cb].z, acc[cb], 0, 0, 0);
        acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.w, b4[cb].w, acc[cb], 0, 0, 0);
      }
    }
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int r = 0; r < 16; ++r) accd[cb][r] += (double)acc[cb][r];
  }
  store_tile<CB>(t, accd, P, lineTotal, nrhoSorted, lineOffSorted, part);
}

// Split-BF16: A = A0 + A1 + A2, B = B0 + B1 + B2; six products per K-step,
// the five small ones (02, 11, 20, 01, 10) accumulated apart from 00 so that
// their rounding stays at their own (2^-8 smaller) scale.
template <int CB>
__global__ __launch_bounds__(64) void k_contract_bf16x6(
    const Tile* __restrict__ tiles, int NrPad, int kchunk, int P, int lineTotal,
    const uint16_t* __restrict__ Msplit, const uint16_t* __restrict__ Bsplit,
    const int32_t* __restrict__ nrhoSorted, const int32_t* __restrict__ lineOffSorted,
    double* __restrict__ part) {
  const Tile t = tiles[blockIdx.x];
  if (t.row0 < 0) return;
  const int lane = threadIdx.x;
  const int hb = lane >> 5;
  const int rr = lane & 31;
  const int ng = NrPad / 8;
  const uint4* arow = (const uint4*)(Msplit + ((size_t)(t.row0 + rr) * ng + hb) * 24);
  const uint4* bcol[CB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb)
    bcol[cb] = (const uint4*)(Bsplit + ((size_t)(t.col0 + 32 * cb + rr) * ng + hb) * 24);
  double accd[CB][16];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb)
#pragma unroll
    for (int r = 0; r < 16; ++r) accd[cb][r] = 0.0;

  for (int ks = t.k0; ks < t.k0 + kchunk; ks += kSubChunk) {
    f32x16 hi[CB], lo[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        hi[cb][r] = 0.f;
        lo[cb][r] = 0.f;
      }
#pragma unroll 2
    for (int k0 = ks; k0 < ks + kSubChunk; k0 += 16) {
      // group index of this lane's 8 nodes: k0/8 + hb (hb folded into the base)
      const uint4* ap = arow + (size_t)(k0 >> 3) * 3;
      const bf16x8 a0 = as_bf16x8(ap[0]);
      const bf16x8 a1 = as_bf16x8(ap[1]);
      const bf16x8 a2 = as_bf16x8(ap[2]);
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const uint4* bp = bcol[cb] + (size_t)(k0 >> 3) * 3;
        const bf16x8 b0 = as_bf16x8(bp[0]);
        const bf16x8 b1 = as_bf16x8(bp[1]);
        const bf16x8 b2 = as_bf16x8(bp[2]);
        lo[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b2, lo[cb], 0, 0, 0);
        lo[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, lo[cb], 0, 0, 0);
        lo[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2, b0, lo[cb], 0, 0, 0);
        lo[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, lo[cb], 0, 0, 0);
        lo[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, lo[cb], 0, 0, 0);
        hi[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, hi[cb], 0, 0, 0);
      }
    }
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int r = 0; r < 16; ++r) accd[cb][r] += (double)hi[cb][r] + (double)lo[cb][r];
  }
  store_tile<CB>(t, accd, P, lineTotal, nrhoSorted, lineOffSorted, part);
}

// --------------------------------------------------------------------------
// Hankel contraction, LDS-staged version.  A workgroup of 4 waves owns a tile
// of 32*rbN rows (rbN <= RB) x 128*CB columns.  The rows of M for the
// current K-block (32 radial nodes) are staged in LDS, double buffered, and
// shared by the 4 waves; each wave streams its own 32*CB screen columns from
// global memory into registers, one K-step ahead.  Per K-step of 16 nodes a
// wave issues 6 * rbN * CB (split) or 8 * rbN * CB (FP32) MFMAs.  Every
// kSubChunk nodes the FP32 matrix-core sums are added to FP64 running sums.
// --------------------------------------------------------------------------
constexpr int kKB = 32;  // radial nodes per LDS stage

template <int RB, int CB>
__device__ __forceinline__ void store_tile_v2(const Tile& t, int wave, const double (*accd)[16],
                                              int P, int lineTotal,
                                              const int32_t* __restrict__ nrhoSorted,
                                              const int32_t* __restrict__ lineOffSorted,
                                              double* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int hb = lane >> 5;
  const int rr = lane & 31;
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const int col = t.col0 + 32 * (CB * wave + cb) + rr;
    const int j = col >> 1;
    const int comp = col & 1;
    if (j >= P || j >= t.pad[0]) continue;  // pad[0]: end of the tile's chunk
    const int nr = nrhoSorted[j];
    double* dst = part + ((size_t)t.kc * lineTotal + lineOffSorted[j]) * 2 + comp;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      if (rb >= t.rbN) break;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = t.row0 + 32 * rb + 8 * (r >> 2) + 4 * hb + (r & 3);
        if (row < nr) dst[(size_t)row * 2] = accd[rb * CB + cb][r];
      }
    }
  }
}

template <int RB, int CB>
__global__ __launch_bounds__(256) void k_contract_bf16x6_lds(
    const Tile* __restrict__ tiles, int NrPad, int kchunk, int P, int lineTotal,
    const uint4* __restrict__ Msplit, const uint4* __restrict__ Bsplit,
    const int32_t* __restrict__ nrhoSorted, const int32_t* __restrict__ lineOffSorted,
    double* __restrict__ part) {
  constexpr int BM = 32 * RB;
  constexpr int KG = kKB / 8;                 // 8-node groups per stage
  constexpr int NFILL = BM * KG * 3;          // uint4 per stage
  constexpr int FILL = (NFILL + 255) / 256;   // per thread
  __shared__ uint4 lds[2][KG][BM][3];
  const Tile t = tiles[blockIdx.x];
  if (t.row0 < 0) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int hb = lane >> 5;
  const int rr = lane & 31;
  const int ng = NrPad / 8;
  const int rowsN = 32 * t.rbN;

  // global -> LDS fill assignment: uint4 f = tid + 256 i -> (row, group, term)
  const uint4* fsrc[FILL];
  int fdst[FILL];
  bool fon[FILL];
#pragma unroll
  for (int i = 0; i < FILL; ++i) {
    const int f = tid + 256 * i;
    const int row = f / (KG * 3);
    const int c = f - row * (KG * 3);
    const int kg = c / 3;
    const int term = c - kg * 3;
    fon[i] = f < NFILL && row < rowsN;
    fsrc[i] = Msplit + ((size_t)(t.row0 + (fon[i] ? row : 0)) * ng + kg) * 3 + term;
    fdst[i] = (kg * BM + row) * 3 + term;
  }
  const uint4* bsrc[CB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb)
    bsrc[cb] = Bsplit + ((size_t)(t.col0 + 32 * (CB * wave + cb) + rr) * ng + hb) * 3;

  double accd[RB * CB][16];
#pragma unroll
  for (int b = 0; b < RB * CB; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) accd[b][r] = 0.0;
  f32x16 hi[RB * CB], lo[RB * CB];
#pragma unroll
  for (int b = 0; b < RB * CB; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      hi[b][r] = 0.f;
      lo[b][r] = 0.f;
    }

  const int kEnd = t.k0 + kchunk;
  uint4 stage[FILL];
  // prologue: stage 0 into buffer 0
#pragma unroll
  for (int i = 0; i < FILL; ++i)
    if (fon[i]) stage[i] = fsrc[i][(size_t)(t.k0 / 8) * 3];
#pragma unroll
  for (int i = 0; i < FILL; ++i)
    if (fon[i]) (&lds[0][0][0][0])[fdst[i]] = stage[i];
  uint4 bq[CB][3];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb)
#pragma unroll
    for (int q = 0; q < 3; ++q) bq[cb][q] = bsrc[cb][(size_t)(t.k0 / 8) * 3 + q];
  __syncthreads();

  int buf = 0;
  for (int kb = t.k0; kb < kEnd; kb += kKB) {
    const bool more = kb + kKB < kEnd;
    if (more) {
#pragma unroll
      for (int i = 0; i < FILL; ++i)
        if (fon[i]) stage[i] = fsrc[i][(size_t)((kb + kKB) / 8) * 3];
    }
#pragma unroll
    for (int s = 0; s < kKB / 16; ++s) {
      const int k = kb + 16 * s;
      // prefetch the next K-step's screen fragments
      uint4 bn[CB][3];
      const bool nextOk = k + 16 < kEnd;
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int q = 0; q < 3; ++q)
          bn[cb][q] = nextOk ? bsrc[cb][(size_t)((k + 16) / 8) * 3 + q] : bq[cb][q];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        if (rb >= t.rbN) break;
        const uint4* ap = &lds[buf][2 * s + hb][32 * rb + rr][0];
        const bf16x8 a0 = as_bf16x8(ap[0]);
        const bf16x8 a1 = as_bf16x8(ap[1]);
        const bf16x8 a2 = as_bf16x8(ap[2]);
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          const int b = rb * CB + cb;
          const bf16x8 b0 = as_bf16x8(bq[cb][0]);
          const bf16x8 b1 = as_bf16x8(bq[cb][1]);
          const bf16x8 b2 = as_bf16x8(bq[cb][2]);
          lo[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b2, lo[b], 0, 0, 0);
          lo[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, lo[b], 0, 0, 0);
          lo[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2, b0, lo[b], 0, 0, 0);
          lo[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, lo[b], 0, 0, 0);
          lo[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, lo[b], 0, 0, 0);
          hi[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, hi[b], 0, 0, 0);
        }
      }
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int q = 0; q < 3; ++q) bq[cb][q] = bn[cb][q];
    }
    if (((kb + kKB - t.k0) % kSubChunk) == 0) {
      flush_fp64(accd, hi, lo);
    }
    if (more) {
#pragma unroll
      for (int i = 0; i < FILL; ++i)
        if (fon[i]) (&lds[buf ^ 1][0][0][0])[fdst[i]] = stage[i];
    }
    __syncthreads();
    buf ^= 1;
  }
  store_tile_v2<RB, CB>(t, wave, accd, P, lineTotal, nrhoSorted, lineOffSorted, part);
}

template <int RB, int CB>
__global__ __launch_bounds__(256) void k_contract_f32_lds(
    const Tile* __restrict__ tiles, int NrPad, int kchunk, int P, int lineTotal,
    const float4* __restrict__ M32, const float4* __restrict__ B32,
    const int32_t* __restrict__ nrhoSorted, const int32_t* __restrict__ lineOffSorted,
    double* __restrict__ part) {
  constexpr int BM = 32 * RB;
  constexpr int KQ = kKB / 4;              // 4-node quads per stage
  constexpr int NFILL = BM * KQ;           // float4 per stage
  constexpr int FILL = (NFILL + 255) / 256;
  __shared__ float4 lds[2][KQ][BM];
  const Tile t = tiles[blockIdx.x];
  if (t.row0 < 0) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int hb = lane >> 5;
  const int rr = lane & 31;
  const int nq = NrPad / 4;
  const int rowsN = 32 * t.rbN;

  const float4* fsrc[FILL];
  int fdst[FILL];
  bool fon[FILL];
#pragma unroll
  for (int i = 0; i < FILL; ++i) {
    const int f = tid + 256 * i;
    const int row = f / KQ;
    const int kq = f - row * KQ;
    fon[i] = f < NFILL && row < rowsN;
    fsrc[i] = M32 + (size_t)(t.row0 + (fon[i] ? row : 0)) * nq + kq;
    fdst[i] = kq * BM + row;
  }
  const float4* bsrc[CB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb)
    bsrc[cb] = B32 + (size_t)(t.col0 + 32 * (CB * wave + cb) + rr) * nq + hb;

  double accd[RB * CB][16];
#pragma unroll
  for (int b = 0; b < RB * CB; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) accd[b][r] = 0.0;
  f32x16 acc[RB * CB];
#pragma unroll
  for (int b = 0; b < RB * CB; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[b][r] = 0.f;

  const int kEnd = t.k0 + kchunk;
  float4 stage[FILL];
#pragma unroll
  for (int i = 0; i < FILL; ++i)
    if (fon[i]) stage[i] = fsrc[i][t.k0 / 4];
#pragma unroll
  for (int i = 0; i < FILL; ++i)
    if (fon[i]) (&lds[0][0][0])[fdst[i]] = stage[i];
  float4 bq[CB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) bq[cb] = bsrc[cb][t.k0 / 4];
  __syncthreads();

  int buf = 0;
  for (int kb = t.k0; kb < kEnd; kb += kKB) {
    const bool more = kb + kKB < kEnd;
    if (more) {
#pragma unroll
      for (int i = 0; i < FILL; ++i)
        if (fon[i]) stage[i] = fsrc[i][(kb + kKB) / 4];
    }
#pragma unroll
    for (int s = 0; s < kKB / 8; ++s) {
      const int k = kb + 8 * s;
      float4 bn[CB];
      const bool nextOk = k + 8 < kEnd;
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) bn[cb] = nextOk ? bsrc[cb][(k + 8) / 4] : bq[cb];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        if (rb >= t.rbN) break;
        const float4 a4 = lds[buf][2 * s + hb][32 * rb + rr];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          const int b = rb * CB + cb;
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.x, bq[cb].x, acc[b], 0, 0, 0);
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.y, bq[cb].y, acc[b], 0, 0, 0);
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.z, bq[cb].z, acc[b], 0, 0, 0);
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.w, bq[cb].w, acc[b], 0, 0, 0);
        }
      }
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) bq[cb] = bn[cb];
    }
    if (((kb + kKB - t.k0) % kSubChunk) == 0) {
#pragma unroll
      for (int b = 0; b < RB * CB; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          accd[b][r] += (double)acc[b][r];
          acc[b][r] = 0.f;
        }
    }
    if (more) {
#pragma unroll
      for (int i = 0; i < FILL; ++i)
        if (fon[i]) (&lds[buf ^ 1][0][0])[fdst[i]] = stage[i];
    }
    __syncthreads();
    buf ^= 1;
  }
  store_tile_v2<RB, CB>(t, wave, accd, P, lineTotal, nrhoSorted, lineOffSorted, part);
}

// --------------------------------------------------------------------------
// Hankel contraction, split-BF16, with an LDS ring filled by direct
// global-to-LDS loads (gfx950 global_load_lds_dwordx4: each lane's 16 bytes
// land at the wave's LDS base + 16 * lane, no VGPRs involved).  A workgroup
// of 4 waves, arranged WR x WC, owns a tile of 32 RBW WR rows x 32 CBW WC
// columns; each wave computes RBW x CBW MFMA blocks of 32 x 32.  One stage is
// one MFMA K-step of 16 radial nodes: the rows of M and the screen columns of
// the tile for those nodes (3 BF16 terms each) are loaded into ring slot
// s % NS while the waves compute from older slots; NS - 1 stages are in
// flight.  Every kSubChunk nodes the FP32 matrix-core sums go to FP64.
//
// Keeping the loads in flight takes two things the plain idioms defeat:
// every slot is its own LDS object, and the slot a stage touches is a
// compile-time constant (the stage loop is unrolled by NS), so the compiler
// can tell that the reads of one slot do not depend on the loads into the
// others; and the workgroup barrier is a bare s_barrier after an explicit
// vmcnt wait for this stage's loads only, since a barrier with a
// workgroup-scope fence waits for every outstanding load.
// --------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  // s_waitcnt with vmcnt = N, expcnt and lgkmcnt left at their maxima
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

template <int WR, int WC, int RBW, int CBW, int NS>
__global__ __launch_bounds__(256) void k_contract_bf16x6_ring(
    const Tile* __restrict__ tiles, int NrPad, int kchunk, int P, int lineTotal,
    const uint4* __restrict__ Msplit, const uint4* __restrict__ Bsplit,
    const int32_t* __restrict__ nrhoSorted, const int32_t* __restrict__ lineOffSorted,
    double* __restrict__ part) {
  constexpr int BM = 32 * RBW * WR;
  constexpr int BN = 32 * CBW * WC;
  constexpr int AU = BM * 2 * 3;            // uint4 of M per stage (2 groups of 8 nodes)
  constexpr int SU = AU + BN * 2 * 3;       // uint4 per stage
  constexpr int LW = (SU + 255) / 256;      // load instructions per wave per stage
  constexpr int SLOT = LW * 256;            // padded slot size (uint4)
  static_assert(NS == 3 || NS == 4, "ring depth");
  static_assert(LW * (NS - 2) < 64, "too many loads in flight for vmcnt");
  __shared__ uint4 ring0[SLOT];
  __shared__ uint4 ring1[SLOT];
  __shared__ uint4 ring2[SLOT];
  __shared__ uint4 ring3[NS == 4 ? SLOT : 1];

  const Tile t = tiles[blockIdx.x];
  if (t.row0 < 0) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave / WC;
  const int wc = wave - wr * WC;
  const int hb = lane >> 5;
  const int rr = lane & 31;
  const int ng = NrPad / 8;
  const int kg0 = t.k0 / 8;

  // this thread's source for ring element u = 256 * l + tid of every stage
  // (stage s adds 2 groups = 6 uint4 to every source)
  const uint4* src[LW];
#pragma unroll
  for (int l = 0; l < LW; ++l) {
    int u = 256 * l + tid;
    if (u >= SU) u = 0;  // padding lanes reload element 0 into the slot's tail
    if (u < AU) {
      const int grp = u / (BM * 3);
      const int row = (u / 3) % BM;
      const int term = u % 3;
      src[l] = Msplit + ((size_t)(t.row0 + row) * ng + kg0 + grp) * 3 + term;
    } else {
      const int v = u - AU;
      const int grp = v / (BN * 3);
      const int col = (v / 3) % BN;
      const int term = v % 3;
      src[l] = Bsplit + ((size_t)(t.col0 + col) * ng + kg0 + grp) * 3 + term;
    }
  }
  const int nst = kchunk / 16;  // a multiple of 16

  double accd[RBW * CBW][16];
  f32x16 hi[RBW * CBW], lo[RBW * CBW];
#pragma unroll
  for (int b = 0; b < RBW * CBW; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      accd[b][r] = 0.0;
      hi[b][r] = 0.f;
      lo[b][r] = 0.f;
    }
  const int rbBase = wr * RBW;

  auto slot_of = [&](auto kc) -> uint4* {
    constexpr int K = decltype(kc)::value;
    if constexpr (K == 0) return ring0;
    else if constexpr (K == 1) return ring1;
    else if constexpr (K == 2) return ring2;
    else return ring3;
  };
  auto issue = [&](auto kc, int stage) {
    uint4* slot = slot_of(kc);
#pragma unroll
    for (int l = 0; l < LW; ++l)
      __builtin_amdgcn_global_load_lds((const void*)(src[l] + (size_t)stage * 6),
                                       (__attribute__((address_space(3))) void*)(slot + 256 * l +
                                                                                 64 * wave),
                                       16, 0, 0);
  };
  // workgroup barrier without a memory fence; the empty asm statements keep
  // the compiler from moving LDS accesses across it
  auto barrier = [&]() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };
  auto step = [&](auto kc, int s) {
    constexpr int K = decltype(kc)::value;
    constexpr int KN = (K + NS - 1) % NS;  // slot of stage s + NS - 1
    // this wave's loads of stage s have landed; after the barrier so have
    // every wave's, and every wave is done reading slot KN (stage s - 1)
    if (s + NS - 2 < nst)
      wait_vmcnt<LW * (NS - 2)>();
    else
      wait_vmcnt<0>();
    barrier();
    if (s + NS - 1 < nst) issue(std::integral_constant<int, KN>{}, s + NS - 1);
    const uint4* slot = slot_of(kc);
    bf16x8 bq[CBW][3];
#pragma unroll
    for (int cb = 0; cb < CBW; ++cb) {
      const uint4* bp = slot + AU + (hb * BN + wc * 32 * CBW + cb * 32 + rr) * 3;
      bq[cb][0] = as_bf16x8(bp[0]);
      bq[cb][1] = as_bf16x8(bp[1]);
      bq[cb][2] = as_bf16x8(bp[2]);
    }
    bf16x8 aq[RBW][3];
#pragma unroll
    for (int rb = 0; rb < RBW; ++rb) {
      const uint4* ap = slot + (hb * BM + (rbBase + rb) * 32 + rr) * 3;
      aq[rb][0] = as_bf16x8(ap[0]);
      aq[rb][1] = as_bf16x8(ap[1]);
      aq[rb][2] = as_bf16x8(ap[2]);
    }
    // products interleaved over the output blocks so consecutive MFMAs are
    // independent; row blocks past the tile's last row compute on padded
    // rows of M and are not stored
    mfma_split6<RBW, CBW>(aq, bq, lo, hi);
    if (((s + 1) * 16) % kSubChunk == 0) {
      flush_fp64(accd, hi, lo);
    }
  };

  issue(std::integral_constant<int, 0>{}, 0);
  issue(std::integral_constant<int, 1>{}, 1);
  if constexpr (NS == 4) {
    issue(std::integral_constant<int, 2>{}, 2);
    for (int s0 = 0; s0 < nst; s0 += 4) {
      step(std::integral_constant<int, 0>{}, s0);
      step(std::integral_constant<int, 1>{}, s0 + 1);
      step(std::integral_constant<int, 2>{}, s0 + 2);
      step(std::integral_constant<int, 3>{}, s0 + 3);
    }
  } else {
    for (int s0 = 0; s0 < nst; s0 += 3) {
      step(std::integral_constant<int, 0>{}, s0);
      if (s0 + 1 < nst) step(std::integral_constant<int, 1>{}, s0 + 1);
      if (s0 + 2 < nst) step(std::integral_constant<int, 2>{}, s0 + 2);
    }
  }

  // store: block (rb, cb) of this wave
#pragma unroll
  for (int cb = 0; cb < CBW; ++cb) {
    const int col = t.col0 + wc * 32 * CBW + cb * 32 + rr;
    const int j = col >> 1;
    const int comp = col & 1;
    if (j >= P || j >= t.pad[0]) continue;
    const int nr = nrhoSorted[j];
    double* dst = part + ((size_t)t.kc * lineTotal + lineOffSorted[j]) * 2 + comp;
#pragma unroll
    for (int rb = 0; rb < RBW; ++rb) {
      if (rbBase + rb >= t.rbN) break;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = t.row0 + (rbBase + rb) * 32 + 8 * (r >> 2) + 4 * hb + (r & 3);
        if (row < nr) dst[(size_t)row * 2] = accd[rb * CBW + cb][r];
      }
    }
  }
}

// --------------------------------------------------------------------------
// The same ring with FP32 operands: M32 rows and FP32 screen columns (4 bytes
// per value instead of 3 BF16 terms) are staged, and every lane splits its
// 8 values into three BF16 terms after reading them from LDS.  The split of
// an FP32 value is exact: x = t0 + t1 + t2 with t0 = bf16(x),
// t1 = bf16(x - t0), t2 = x - t0 - t1 (at most 8 significant bits left).
// A stage holds 16 nodes of every row and column, 64 bytes each, as four
// 16-byte quarters; quarter q of row r sits at slot position 4 r + (q ^ s),
// s = (r / 4) % 4, so that the 16-byte reads of 16 consecutive rows fall in
// distinct LDS banks.  With 4 bytes a value a slot is small enough for an
// 8-stage ring (7 stages in flight: measured 0.55 ms against 0.63 ms with 4
// on the batch workload).  The workgroup has WR x WC waves (4 or 8); with 8
// waves of 32 x 64 each, two waves share a SIMD.  A stage that is not a
// whole number of load rounds for the workgroup ends with a partial round
// issued by the first RW waves only, and each wave waits on its own count.
// --------------------------------------------------------------------------
// Two values rounded to BF16 (nearest even) in one packed conversion: a in
// the low half, b in the high half.
__device__ __forceinline__ uint32_t pk_bf16(float a, float b) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  typedef float f32x2v __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2v){a, b}, bf16x2));
}
// Values are split in pairs: each packed BF16 pair is widened back to FP32
// by a shift (low half) or a mask (high half) to form the residuals, so each
// term costs one conversion per two values.
__device__ __forceinline__ void split_bf16x3(const float4& lo4, const float4& hi4, bf16x8& t0,
                                             bf16x8& t1, bf16x8& t2) {
  typedef uint32_t u32x4v __attribute__((ext_vector_type(4)));
  const float x[8] = {lo4.x, lo4.y, lo4.z, lo4.w, hi4.x, hi4.y, hi4.z, hi4.w};
  u32x4v p0, p1, p2;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const float xa = x[2 * e], xb = x[2 * e + 1];
    const uint32_t a = pk_bf16(xa, xb);
    const float ra = xa - __uint_as_float(a << 16);
    const float rb = xb - __uint_as_float(a & 0xffff0000u);
    const uint32_t b = pk_bf16(ra, rb);
    const float sa = ra - __uint_as_float(b << 16);
    const float sb = rb - __uint_as_float(b & 0xffff0000u);
    p0[e] = a;
    p1[e] = b;
    p2[e] = pk_bf16(sa, sb);
  }
  t0 = __builtin_bit_cast(bf16x8, p0);
  t1 = __builtin_bit_cast(bf16x8, p1);
  t2 = __builtin_bit_cast(bf16x8, p2);
}

template <int WR, int WC, int RBW, int CBW, int NS>
__global__ __launch_bounds__(64 * WR * WC) void k_contract_bf16x6_ringf(
    const Tile* __restrict__ tiles, int NrPad, int kchunk, int P, int lineTotal,
    const float* __restrict__ M32, const float* __restrict__ B32,
    const int32_t* __restrict__ nrhoSorted, const int32_t* __restrict__ lineOffSorted,
    double* __restrict__ part) {
  constexpr int BM = 32 * RBW * WR;
  constexpr int BN = 32 * CBW * WC;
  constexpr int NT = 64 * WR * WC;          // threads
  constexpr int AU = BM * 4;                // 16-byte quarters of M per stage
  constexpr int SU = AU + BN * 4;           // quarters per stage
  // LF load rounds of every wave, then one more by the first RW waves
  constexpr int LF = SU / NT;
  constexpr int RW = (SU - LF * NT) / 64;
  constexpr int LW = LF + (RW > 0 ? 1 : 0);
  constexpr int SLOT = SU;
  static_assert(SU % 64 == 0, "whole waves of quarters");
  static_assert(LW * (NS - 2) < 64, "too many loads in flight for vmcnt");
  static_assert(NS == 4 || NS == 8, "ring depth");
  __shared__ float4 ring0[SLOT];
  __shared__ float4 ring1[SLOT];
  __shared__ float4 ring2[SLOT];
  __shared__ float4 ring3[SLOT];
  __shared__ float4 ring4[NS > 4 ? SLOT : 1];
  __shared__ float4 ring5[NS > 4 ? SLOT : 1];
  __shared__ float4 ring6[NS > 4 ? SLOT : 1];
  __shared__ float4 ring7[NS > 4 ? SLOT : 1];

  const Tile t = tiles[blockIdx.x];
  if (t.row0 < 0) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave / WC;
  const int wc = wave - wr * WC;
  const int hb = lane >> 5;
  const int rr = lane & 31;

  // source of slot position u = NT l + tid: position 4 r + q' holds quarter
  // q' ^ ((r / 4) % 4) of row (or column) r; stage s adds 16 nodes
  const float* src[LW];
#pragma unroll
  for (int l = 0; l < LW; ++l) {
    int u = NT * l + tid;
    if (u >= SU) u = 0;  // waves past the last partial round: never issued
    if (u < AU) {
      const int r = u >> 2;
      const int qd = (u & 3) ^ ((r >> 2) & 3);
      src[l] = M32 + (size_t)(t.row0 + r) * NrPad + t.k0 + 4 * qd;
    } else {
      const int c = (u - AU) >> 2;
      const int qd = ((u - AU) & 3) ^ ((c >> 2) & 3);
      src[l] = B32 + (size_t)(t.col0 + c) * NrPad + t.k0 + 4 * qd;
    }
  }
  const int nst = kchunk / 16;  // a multiple of 16

  double accd[RBW * CBW][16];
  f32x16 hi[RBW * CBW], lo[RBW * CBW];
#pragma unroll
  for (int b = 0; b < RBW * CBW; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      accd[b][r] = 0.0;
      hi[b][r] = 0.f;
      lo[b][r] = 0.f;
    }
  const int rbBase = wr * RBW;

  auto slot_of = [&](auto kc) -> float4* {
    constexpr int K = decltype(kc)::value;
    if constexpr (K == 0) return ring0;
    else if constexpr (K == 1) return ring1;
    else if constexpr (K == 2) return ring2;
    else if constexpr (K == 3) return ring3;
    else if constexpr (K == 4) return ring4;
    else if constexpr (K == 5) return ring5;
    else if constexpr (K == 6) return ring6;
    else return ring7;
  };
  auto issue = [&](auto kc, int stage) {
    float4* slot = slot_of(kc);
#pragma unroll
    for (int l = 0; l < LW; ++l)
      if (l < LF || wave < RW)  // wave-uniform
        __builtin_amdgcn_global_load_lds((const void*)(src[l] + (size_t)stage * 16),
                                         (__attribute__((address_space(3))) void*)(slot + NT * l +
                                                                                   64 * wave),
                                         16, 0, 0);
  };
  auto barrier = [&]() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };
  // the 8 nodes hb*8 .. hb*8 + 7 of row (or column) r of a slot region
  auto fragment = [&](const float4* region, int r, bf16x8& t0, bf16x8& t1, bf16x8& t2) {
    const int sw = (r >> 2) & 3;
    const float4 a = region[4 * r + ((2 * hb) ^ sw)];
    const float4 b = region[4 * r + ((2 * hb + 1) ^ sw)];
    split_bf16x3(a, b, t0, t1, t2);
  };
  auto step = [&](auto kc, int s) {
    constexpr int K = decltype(kc)::value;
    constexpr int KN = (K + NS - 1) % NS;
    // a wave issues LW loads a stage if it takes part in the partial round,
    // LF otherwise
    if (s + NS - 2 < nst) {
      if (RW == 0 || wave < RW)
        wait_vmcnt<LW * (NS - 2)>();
      else
        wait_vmcnt<LF * (NS - 2)>();
    } else {
      wait_vmcnt<0>();
    }
    barrier();
    if (s + NS - 1 < nst) issue(std::integral_constant<int, KN>{}, s + NS - 1);
    const float4* slot = slot_of(kc);
    bf16x8 bq[CBW][3];
#pragma unroll
    for (int cb = 0; cb < CBW; ++cb)
      fragment(slot + AU, wc * 32 * CBW + cb * 32 + rr, bq[cb][0], bq[cb][1], bq[cb][2]);
    bf16x8 aq[RBW][3];
#pragma unroll
    for (int rb = 0; rb < RBW; ++rb)
      fragment(slot, (rbBase + rb) * 32 + rr, aq[rb][0], aq[rb][1], aq[rb][2]);
    mfma_split6<RBW, CBW>(aq, bq, lo, hi);
    if (((s + 1) * 16) % kSubChunk == 0) {
      flush_fp64(accd, hi, lo);
    }
  };

  issue(std::integral_constant<int, 0>{}, 0);
  issue(std::integral_constant<int, 1>{}, 1);
  issue(std::integral_constant<int, 2>{}, 2);
  if constexpr (NS == 8) {
    issue(std::integral_constant<int, 3>{}, 3);
    issue(std::integral_constant<int, 4>{}, 4);
    issue(std::integral_constant<int, 5>{}, 5);
    issue(std::integral_constant<int, 6>{}, 6);
  }
  for (int s0 = 0; s0 < nst; s0 += NS) {
    step(std::integral_constant<int, 0>{}, s0);
    step(std::integral_constant<int, 1>{}, s0 + 1);
    step(std::integral_constant<int, 2>{}, s0 + 2);
    step(std::integral_constant<int, 3>{}, s0 + 3);
    if constexpr (NS == 8) {
      step(std::integral_constant<int, 4>{}, s0 + 4);
      step(std::integral_constant<int, 5>{}, s0 + 5);
      step(std::integral_constant<int, 6>{}, s0 + 6);
      step(std::integral_constant<int, 7>{}, s0 + 7);
    }
  }

#pragma unroll
  for (int cb = 0; cb < CBW; ++cb) {
    const int col = t.col0 + wc * 32 * CBW + cb * 32 + rr;
    const int j = col >> 1;
    const int comp = col & 1;
    if (j >= P || j >= t.pad[0]) continue;
    const int nr = nrhoSorted[j];
    double* dst = part + ((size_t)t.kc * lineTotal + lineOffSorted[j]) * 2 + comp;
#pragma unroll
    for (int rb = 0; rb < RBW; ++rb) {
      if (rbBase + rb >= t.rbN) break;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = t.row0 + (rbBase + rb) * 32 + 8 * (r >> 2) + 4 * hb + (r & 3);
        if (row < nr) dst[(size_t)row * 2] = accd[rb * CBW + cb][r];
      }
    }
  }
}

// --------------------------------------------------------------------------
// Split-BF16 contraction with M taken as its plan-time BF16 terms (split from
// the FP64 value, node-group-major layout MsplitG[i/8][term][row][8]) and the
// FP32 screen split in registers.  A workgroup of 8 waves computes 64 rows x
// 256 columns; wave w owns columns 32 w .. 32 w + 31 for all 64 rows (two
// 32x32 blocks), so every screen value is split by exactly one wave and no
// wave converts M.  A stage of 16 nodes holds M's terms as [group][term][row]
// (16 bytes a row: consecutive lanes read consecutive LDS quads) and the
// screen columns as four 16-byte quarters each, XOR-swizzled as in the FP32
// ring.  The stage is 22 KB, so 7 stages fit in LDS (6 in flight).  The
// products, their order and the FP64 combine are the other split variants'.
// --------------------------------------------------------------------------
template <int NS>
__global__ __launch_bounds__(512) void k_contract_bf16x6_ringh(
    const Tile* __restrict__ tiles, int NrPad, int rowsPad, int kchunk, int P, int lineTotal,
    const uint4* __restrict__ MsplitG, const float* __restrict__ B32,
    const int32_t* __restrict__ nrhoSorted, const int32_t* __restrict__ lineOffSorted,
    double* __restrict__ part) {
  constexpr int BM = 64, BN = 256, NT = 512, RB = 2;
  constexpr int AU = 2 * 3 * BM;          // uint4 of M terms per stage
  constexpr int SU = AU + BN * 4;         // plus the screen quarters
  constexpr int LF = SU / NT;             // full load rounds of every wave
  constexpr int RW = (SU - LF * NT) / 64; // waves issuing one more round
  constexpr int LW = LF + (RW > 0 ? 1 : 0);
  static_assert(SU % 64 == 0 && AU % 64 == 0, "whole waves per region");
  static_assert(LW * (NS - 2) < 64, "too many loads in flight for vmcnt");
  static_assert(NS == 7, "ring depth");
  __shared__ uint4 ring0[SU];
  __shared__ uint4 ring1[SU];
  __shared__ uint4 ring2[SU];
  __shared__ uint4 ring3[SU];
  __shared__ uint4 ring4[SU];
  __shared__ uint4 ring5[SU];
  __shared__ uint4 ring6[SU];

  const Tile t = tiles[blockIdx.x];
  if (t.row0 < 0) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int hb = lane >> 5;
  const int rr = lane & 31;

  // source of slot position u = NT l + tid and its advance per stage (bytes)
  const char* src[LW];
  int adv[LW];
#pragma unroll
  for (int l = 0; l < LW; ++l) {
    int u = NT * l + tid;
    if (u >= SU) u = 0;  // waves past the last partial round: never issued
    if (u < AU) {
      const int grp = u / (3 * BM);
      const int term = (u / BM) % 3;
      const int row = u % BM;
      src[l] = (const char*)(MsplitG + ((size_t)(t.k0 / 8 + grp) * 3 + term) * rowsPad + t.row0 +
                             row);
      adv[l] = 2 * 3 * rowsPad * 16;
    } else {
      const int c = (u - AU) >> 2;
      const int qd = ((u - AU) & 3) ^ ((c >> 2) & 3);
      src[l] = (const char*)(B32 + (size_t)(t.col0 + c) * NrPad + t.k0 + 4 * qd);
      adv[l] = 64;
    }
  }
  const int nst = kchunk / 16;  // a multiple of 16

  double accd[RB][16];
  f32x16 hi[RB], lo[RB];
#pragma unroll
  for (int b = 0; b < RB; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      accd[b][r] = 0.0;
      hi[b][r] = 0.f;
      lo[b][r] = 0.f;
    }

  auto slot_of = [&](auto kc) -> uint4* {
    constexpr int K = decltype(kc)::value;
    if constexpr (K == 0) return ring0;
    else if constexpr (K == 1) return ring1;
    else if constexpr (K == 2) return ring2;
    else if constexpr (K == 3) return ring3;
    else if constexpr (K == 4) return ring4;
    else if constexpr (K == 5) return ring5;
    else return ring6;
  };
  auto issue = [&](auto kc, int stage) {
    uint4* slot = slot_of(kc);
#pragma unroll
    for (int l = 0; l < LW; ++l)
      if (l < LF || wave < RW)  // wave-uniform
        __builtin_amdgcn_global_load_lds((const void*)(src[l] + (size_t)stage * adv[l]),
                                         (__attribute__((address_space(3))) void*)(slot + NT * l +
                                                                                   64 * wave),
                                         16, 0, 0);
  };
  auto barrier = [&]() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };
  const int col = 32 * wave + rr;  // this lane's column in the tile
  const int sw = (col >> 2) & 3;
  auto step = [&](auto kc, int s) {
    constexpr int K = decltype(kc)::value;
    constexpr int KN = (K + NS - 1) % NS;
    if (s + NS - 2 < nst) {
      if (RW == 0 || wave < RW)
        wait_vmcnt<LW * (NS - 2)>();
      else
        wait_vmcnt<LF * (NS - 2)>();
    } else {
      wait_vmcnt<0>();
    }
    barrier();
    if (s + NS - 1 < nst) issue(std::integral_constant<int, KN>{}, s + NS - 1);
    const uint4* slot = slot_of(kc);
    // the 8 nodes hb*8 .. hb*8 + 7 of this lane's column, split into terms
    bf16x8 bq[1][3];
    {
      const float4* bs = (const float4*)(slot + AU);
      const float4 a = bs[4 * col + ((2 * hb) ^ sw)];
      const float4 b = bs[4 * col + ((2 * hb + 1) ^ sw)];
      split_bf16x3(a, b, bq[0][0], bq[0][1], bq[0][2]);
    }
    bf16x8 aq[RB][3];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int term = 0; term < 3; ++term)
        aq[rb][term] = as_bf16x8(slot[(hb * 3 + term) * BM + rb * 32 + rr]);
    mfma_split6<RB, 1>(aq, bq, lo, hi);
    if (((s + 1) * 16) % kSubChunk == 0) {
      flush_fp64(accd, hi, lo);
    }
  };

  issue(std::integral_constant<int, 0>{}, 0);
  issue(std::integral_constant<int, 1>{}, 1);
  issue(std::integral_constant<int, 2>{}, 2);
  issue(std::integral_constant<int, 3>{}, 3);
  issue(std::integral_constant<int, 4>{}, 4);
  issue(std::integral_constant<int, 5>{}, 5);
  // nst is a multiple of 16: two full rounds of the 7 slots, then a tail
  int s0 = 0;
  for (; s0 + NS <= nst; s0 += NS) {
    step(std::integral_constant<int, 0>{}, s0);
    step(std::integral_constant<int, 1>{}, s0 + 1);
    step(std::integral_constant<int, 2>{}, s0 + 2);
    step(std::integral_constant<int, 3>{}, s0 + 3);
    step(std::integral_constant<int, 4>{}, s0 + 4);
    step(std::integral_constant<int, 5>{}, s0 + 5);
    step(std::integral_constant<int, 6>{}, s0 + 6);
  }
  // the remaining nst - s0 < 7 stages, starting at slot 0
  if (s0 < nst) step(std::integral_constant<int, 0>{}, s0);
  if (s0 + 1 < nst) step(std::integral_constant<int, 1>{}, s0 + 1);
  if (s0 + 2 < nst) step(std::integral_constant<int, 2>{}, s0 + 2);
  if (s0 + 3 < nst) step(std::integral_constant<int, 3>{}, s0 + 3);
  if (s0 + 4 < nst) step(std::integral_constant<int, 4>{}, s0 + 4);
  if (s0 + 5 < nst) step(std::integral_constant<int, 5>{}, s0 + 5);

  const int gcol = t.col0 + col;
  const int j = gcol >> 1;
  const int comp = gcol & 1;
  if (j >= P || j >= t.pad[0]) return;
  const int nr = nrhoSorted[j];
  double* dst = part + ((size_t)t.kc * lineTotal + lineOffSorted[j]) * 2 + comp;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    if (rb >= t.rbN) break;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = t.row0 + rb * 32 + 8 * (r >> 2) + 4 * hb + (r & 3);
      if (row < nr) dst[(size_t)row * 2] = accd[rb][r];
    }
  }
}

// --------------------------------------------------------------------------
// The tile, wave mapping and products of the ring above, with the operands
// staged through registers and a lighter running sum.  Each thread loads its
// share of a stage with 16-byte global loads three stages ahead and writes
// it to one of three LDS slots one stage ahead: this path streams the tile
// operands faster than the direct-to-LDS loads.  The registers it needs come
// from the accumulation.  The 00 product still sums on the matrix cores in
// FP32 over kSubChunk nodes, but the running sum is an FP32 pair (big, comp)
// instead of an FP64 value: at each flush big + hi is formed with an exact
// two-sum and its rounding error added to comp, and the five small products
// accumulate on the matrix cores straight into comp (they are 2^-8 of the
// 00 product and smaller, comp's own rounding is below the pair's).  Three
// registers per output instead of four; the result is big + comp in FP64.
// --------------------------------------------------------------------------
// f(integral_constant<int, 0>) ... f(integral_constant<int, N - 1>), in order.
template <int N, class F>
__device__ __forceinline__ void unroll_steps(F&& f) {
  if constexpr (N > 0) {
    unroll_steps<N - 1>(f);
    f(std::integral_constant<int, N - 1>{});
  }
}

__device__ __forceinline__ void two_sum_into(float& big, float& comp, float hi) {
  const float s = big + hi;
  const float bp = s - big;
  const float e = (big - (s - bp)) + (hi - bp);
  big = s;
  comp += e;
}

// End of a sub-chunk in the two-sum variants: the FP32 sum of the 00
// product (hi) is added to the pair (big, comp) with an exact two-sum and
// starts again from zero; comp also holds the small products.
template <int NB>
__device__ __forceinline__ void flush_two_sum(float (&big)[NB][16], f32x16 (&comp)[NB],
                                              f32x16 (&hi)[NB]) {
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      float c = comp[b][r];
      two_sum_into(big[b][r], c, hi[b][r]);
      comp[b][r] = c;
      hi[b][r] = 0.f;
    }
}

__global__ __launch_bounds__(512) void k_contract_bf16x6_ringr(
    const Tile* __restrict__ tiles, int NrPad, int rowsPad, int kchunk, int P, int lineTotal,
    const uint4* __restrict__ MsplitG, const float* __restrict__ B32,
    const int32_t* __restrict__ nrhoSorted, const int32_t* __restrict__ lineOffSorted,
    double* __restrict__ part) {
  constexpr int BM = 64, BN = 256, NT = 512, RB = 2;
  constexpr int AU = 2 * 3 * BM;          // uint4 of M terms per stage
  constexpr int SU = AU + BN * 4;         // plus the screen quarters
  constexpr int LF = SU / NT;             // full load rounds of every wave
  constexpr int RW = (SU - LF * NT) / 64; // waves loading one more item
  constexpr int LW = LF + (RW > 0 ? 1 : 0);
  static_assert(SU % 64 == 0 && AU % 64 == 0, "whole waves per region");
  // a slot holds LW full rounds, so that every thread stores its LW items
  // (the waves past the last partial round into the tail, never read)
  __shared__ uint4 slot0[NT * LW];
  __shared__ uint4 slot1[NT * LW];
  __shared__ uint4 slot2[NT * LW];

  const Tile t = tiles[blockIdx.x];
  if (t.row0 < 0) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int hb = lane >> 5;
  const int rr = lane & 31;

  // item u = NT l + tid of a stage: its source and its advance per stage
  const char* src[LW];
  int adv[LW];
#pragma unroll
  for (int l = 0; l < LW; ++l) {
    int u = NT * l + tid;
    if (u >= SU) u = 0;  // waves past the last partial round: loaded, not stored
    if (u < AU) {
      const int grp = u / (3 * BM);
      const int term = (u / BM) % 3;
      const int row = u % BM;
      src[l] = (const char*)(MsplitG + ((size_t)(t.k0 / 8 + grp) * 3 + term) * rowsPad + t.row0 +
                             row);
      adv[l] = 2 * 3 * rowsPad * 16;
    } else {
      const int c = (u - AU) >> 2;
      const int qd = ((u - AU) & 3) ^ ((c >> 2) & 3);
      src[l] = (const char*)(B32 + (size_t)(t.col0 + c) * NrPad + t.k0 + 4 * qd);
      adv[l] = 64;
    }
  }
  const int nst = kchunk / 16;  // a multiple of 16

  f32x16 hi[RB], comp[RB];
  float big[RB][16];
#pragma unroll
  for (int b = 0; b < RB; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      hi[b][r] = 0.f;
      comp[b][r] = 0.f;
      big[b][r] = 0.f;
    }

  // the three register sets, named directly (a pointer to them would put
  // them in scratch memory)
  uint4 rg0[LW], rg1[LW], rg2[LW];
  auto slot_of = [&](auto kc) __attribute__((always_inline)) -> uint4* {
    constexpr int K = decltype(kc)::value;
    if constexpr (K == 0) return slot0;
    else if constexpr (K == 1) return slot1;
    else return slot2;
  };
  // Every wave issues LW loads and LW LDS stores per stage,
  // unconditionally: the compiler's load counting then sees the same number
  // of loads between a register set's load and its use on every path (a
  // conditional load makes it wait for all of them), and a step has no
  // branch to cut its scheduling.  The waves past the last partial round
  // load item 0's source again and store it past the stage; the stages past
  // the end are clamped to the last one and never read.
  auto load = [&](auto kc, int stage) __attribute__((always_inline)) {
    constexpr int K = decltype(kc)::value;
#pragma unroll
    for (int l = 0; l < LW; ++l) {
      const uint4 v = *(const uint4*)(src[l] + (size_t)stage * adv[l]);
      if constexpr (K == 0) rg0[l] = v;
      else if constexpr (K == 1) rg1[l] = v;
      else rg2[l] = v;
    }
  };
  auto store = [&](auto kc) __attribute__((always_inline)) {
    constexpr int K = decltype(kc)::value;
    uint4* slot = slot_of(kc);
#pragma unroll
    for (int l = 0; l < LW; ++l) {
      if constexpr (K == 0) slot[NT * l + tid] = rg0[l];
      else if constexpr (K == 1) slot[NT * l + tid] = rg1[l];
      else slot[NT * l + tid] = rg2[l];
    }
  };
  auto barrier = [&]() __attribute__((always_inline)) {
    // the stage's LDS writes are complete; register loads stay in flight
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0) only
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };
  const int col = 32 * wave + rr;  // this lane's column in the tile
  const int sw = (col >> 2) & 3;
  // The lane's 8 screen values of a stage, split into terms: two sets
  // alternate, so that stage s + 1's values are read and split while the
  // MFMAs of stage s run.  M's terms need no arithmetic and are read for the
  // current stage only.
  bf16x8 bq0[1][3], bq1[1][3], aq[RB][3];
  auto read_b = [&](auto kc, auto fc) __attribute__((always_inline)) {
    constexpr int F = decltype(fc)::value;
    const float4* bs = (const float4*)(slot_of(kc) + AU);
    const float4 x = bs[4 * col + ((2 * hb) ^ sw)];
    const float4 y = bs[4 * col + ((2 * hb + 1) ^ sw)];
    if constexpr (F == 0) split_bf16x3(x, y, bq0[0][0], bq0[0][1], bq0[0][2]);
    else split_bf16x3(x, y, bq1[0][0], bq1[0][1], bq1[0][2]);
  };
  auto read_a = [&](auto kc) __attribute__((always_inline)) {
    const uint4* slot = slot_of(kc);
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int term = 0; term < 3; ++term)
        aq[rb][term] = as_bf16x8(slot[(hb * 3 + term) * BM + rb * 32 + rr]);
  };
  auto mfma = [&](auto fc) __attribute__((always_inline)) {
    constexpr int F = decltype(fc)::value;
    auto& bq = F == 0 ? bq0 : bq1;
    mfma_split6<RB, 1>(aq, bq, comp, hi);
  };
  // Step s (K = s mod 24; slot and register set s mod 3, screen terms
  // s mod 2, flush every 8 steps): stage s + 1 goes from its registers to
  // its slot and the registers take stage s + 4; after the barrier both
  // stage s and stage s + 1 are in LDS, so stage s + 1's screen values are
  // read and split while the MFMAs of stage s (on values split one step
  // earlier) run.  A slot is rewritten two steps after its last read, past
  // a barrier.  The loop is unrolled over 24 steps so that every step is
  // straight-line code (no branch to keep the split apart from the MFMAs):
  // the last steps store, load and split a clamped stage they never use.
  auto step = [&](auto kc, int s) __attribute__((always_inline)) {
    constexpr int K = decltype(kc)::value;
    constexpr int SN = (K + 1) % 3;
    constexpr int FC = K % 2, FN = 1 - FC;
    store(std::integral_constant<int, SN>{});
    load(std::integral_constant<int, SN>{}, min(s + 4, nst - 1));
    barrier();
    read_a(std::integral_constant<int, K % 3>{});
    read_b(std::integral_constant<int, SN>{}, std::integral_constant<int, FN>{});
    mfma(std::integral_constant<int, FC>{});
    if constexpr ((K + 1) % (kSubChunk / 16) == 0) {
      flush_two_sum(big, comp, hi);
    }
  };
  static_assert(24 % (kSubChunk / 16) == 0, "flush period divides the unrolled steps");

  load(std::integral_constant<int, 0>{}, 0);
  load(std::integral_constant<int, 1>{}, 1);
  load(std::integral_constant<int, 2>{}, 2);
  store(std::integral_constant<int, 0>{});
  load(std::integral_constant<int, 0>{}, 3);
  barrier();
  read_b(std::integral_constant<int, 0>{}, std::integral_constant<int, 0>{});
  int s0 = 0;
  for (; s0 + 24 <= nst; s0 += 24)
    unroll_steps<24>([&](auto kc) __attribute__((always_inline)) { step(kc, s0 + decltype(kc)::value); });
  unroll_steps<23>([&](auto kc) __attribute__((always_inline)) {
    if (s0 + decltype(kc)::value < nst) step(kc, s0 + decltype(kc)::value);
  });

  const int gcol = t.col0 + col;
  const int j = gcol >> 1;
  const int cmp = gcol & 1;
  if (j >= P || j >= t.pad[0]) return;
  const int nr = nrhoSorted[j];
  double* dst = part + ((size_t)t.kc * lineTotal + lineOffSorted[j]) * 2 + cmp;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    if (rb >= t.rbN) break;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = t.row0 + rb * 32 + 8 * (r >> 2) + 4 * hb + (r & 3);
      if (row < nr) dst[(size_t)row * 2] = (double)big[rb][r] + (double)comp[rb][r];
    }
  }
}

// --------------------------------------------------------------------------
// The tile, wave mapping and products of the kernel above, with the waves
// loosely coupled and a cheaper running sum.  The 00 product's FP32 sum over
// each 128-node sub-chunk goes into an FP64 running sum (a conversion and an
// add per output, against seven operations for the two-sum); the five small
// products stay in one FP32 accumulator for the whole K-chunk, where their
// rounding (2^-24 of a sum already 2^-8 down) is far below the sub-chunk
// sums' (emulated on the CPU: the same error as the FP64 and two-sum
// combines, 2.2e-8; about 6% faster than the two-sum here).  The screen,
// written node-group-major for this kernel (k_screen_f32_groups), goes
// straight from global
// memory into the registers of the lane that uses it (a lane owns one column
// and 8 nodes of each 16-node stage), four stages ahead, so it needs neither
// LDS nor a barrier.  In the node-group-major layout a wave's load covers 32
// adjacent columns' 64 bytes; the column-major layout scatters them NrPad
// floats apart, and the same kernel on it took 0.30 ms against 0.25.  Only
// M's terms, which all 8 waves share, go through LDS: every thread loads one
// 16-byte item of a stage into registers three stages before it writes it
// to a ring of 8 slots, 4 stages before the stage is used, and the
// workgroup meets at a barrier once every 4 stages.  Between barriers the
// waves drift apart, so one wave's split and loads can partly overlap
// another's MFMAs on the same SIMD (measured: matrix and VALU work of two
// waves on one SIMD overlap only in part, and within one wave not at all).
// Stage t is written at step t - 4 and read at step t: a barrier ends one of
// the steps t - 4 .. t - 1, after the write (RAW); its slot was last read at
// step t - 8, and a barrier ends one of the steps t - 8 .. t - 5 (WAR).  No
// direct-to-LDS loads: the compiler's load counting stays exact.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(512) void k_contract_bf16x6_ringw(
    const Tile* __restrict__ tiles, int colsPad, int rowsPad, int kchunk, int P, int lineTotal,
    const uint4* __restrict__ MsplitG, const float* __restrict__ B32,
    const int32_t* __restrict__ nrhoSorted, const int32_t* __restrict__ lineOffSorted,
    double* __restrict__ part) {
  constexpr int BM = 64, NT = 512, RB = 2;
  constexpr int AU = 2 * 3 * BM;  // uint4 of M terms per stage (384)
  constexpr int NSL = 8;          // M slots
  constexpr int AHEAD = 4;        // stages between a slot's write and its read
  constexpr int PERIOD = 4;       // stages per barrier
  static_assert(AHEAD >= PERIOD && NSL >= AHEAD + PERIOD, "ring arithmetic");
  // one uint4 per thread per stage: the waves past the M terms store item 0
  // again into the slot's tail, never read
  __shared__ uint4 ringA[NSL][NT];

  const Tile t = tiles[blockIdx.x];
  if (t.row0 < 0) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int hb = lane >> 5;
  const int rr = lane & 31;
  const int nst = kchunk / 16;  // a multiple of 16

  // M terms: item u = tid of a stage and its advance per stage (bytes)
  const char* srcA;
  {
    const int u = tid < AU ? tid : 0;
    const int grp = u / (3 * BM);
    const int term = (u / BM) % 3;
    const int row = u % BM;
    srcA = (const char*)(MsplitG + ((size_t)(t.k0 / 8 + grp) * 3 + term) * rowsPad + t.row0 + row);
  }
  const size_t advA = (size_t)2 * 3 * rowsPad * 16;
  // this lane's screen column, nodes hb * 8 .. hb * 8 + 7 of each stage, in
  // the node-group-major screen (a stage of all columns is one contiguous
  // block, so a wave's load covers 32 columns' 64 bytes side by side)
  const int col = 32 * wave + rr;
  const float4* srcB =
      (const float4*)(B32 + ((size_t)(t.k0 / 16) * colsPad + t.col0 + col) * 16 + 8 * hb);
  const size_t advB = (size_t)colsPad * 4;  // float4 per stage

  // hi: the 00 product over the current sub-chunk (FP32); lo: the five small
  // products over the whole K-chunk (FP32, 2^-8 of hi and smaller); sumd: the
  // running sum of the sub-chunks' hi (FP64)
  f32x16 hi[RB], lo[RB];
  double sumd[RB][16];
#pragma unroll
  for (int b = 0; b < RB; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      hi[b][r] = 0.f;
      lo[b][r] = 0.f;
      sumd[b][r] = 0.0;
    }

  // register sets, named directly: M items three stages ahead of their
  // LDS write, raw screen values four stages ahead of their split
  uint4 ra0, ra1, ra2;
  float4 b0x, b0y, b1x, b1y, b2x, b2y, b3x, b3y;
  auto load_a = [&](auto kc, int stage) __attribute__((always_inline)) {
    constexpr int K = decltype(kc)::value;
    const uint4 v = *(const uint4*)(srcA + (size_t)stage * advA);
    if constexpr (K == 0) ra0 = v;
    else if constexpr (K == 1) ra1 = v;
    else ra2 = v;
  };
  auto store_a = [&](auto kc, int slotIdx) __attribute__((always_inline)) {
    constexpr int K = decltype(kc)::value;
    if constexpr (K == 0) ringA[slotIdx][tid] = ra0;
    else if constexpr (K == 1) ringA[slotIdx][tid] = ra1;
    else ringA[slotIdx][tid] = ra2;
  };
  auto load_b = [&](auto kc, int stage) __attribute__((always_inline)) {
    constexpr int K = decltype(kc)::value;
    const float4 x = srcB[advB * stage];
    const float4 y = srcB[advB * stage + 1];
    if constexpr (K == 0) { b0x = x; b0y = y; }
    else if constexpr (K == 1) { b1x = x; b1y = y; }
    else if constexpr (K == 2) { b2x = x; b2y = y; }
    else { b3x = x; b3y = y; }
  };
  auto barrier = [&]() __attribute__((always_inline)) {
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): this wave's LDS writes and reads
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };

  // Step s (K = s mod 24): the M item of stage s + 4 goes from its
  // registers to its slot and the registers take stage s + 7; the raw
  // screen values of stage s are split and their registers take stage
  // s + 4; then the MFMAs of stage s.
  auto step = [&](auto kc, int s) __attribute__((always_inline)) {
    constexpr int K = decltype(kc)::value;
    constexpr int SA = K % 3, SB = K % 4;
    // nothing moves across a step boundary: left free over the 4 steps
    // between barriers, the scheduler sinks each load next to its use
    __builtin_amdgcn_sched_barrier(0);
    store_a(std::integral_constant<int, SA>{}, (K + AHEAD) % NSL);
    load_a(std::integral_constant<int, SA>{}, min(s + AHEAD + 3, nst - 1));
    bf16x8 bq[1][3];
    if constexpr (SB == 0) split_bf16x3(b0x, b0y, bq[0][0], bq[0][1], bq[0][2]);
    else if constexpr (SB == 1) split_bf16x3(b1x, b1y, bq[0][0], bq[0][1], bq[0][2]);
    else if constexpr (SB == 2) split_bf16x3(b2x, b2y, bq[0][0], bq[0][1], bq[0][2]);
    else split_bf16x3(b3x, b3y, bq[0][0], bq[0][1], bq[0][2]);
    load_b(std::integral_constant<int, SB>{}, min(s + 4, nst - 1));
    const uint4* slot = ringA[K % NSL];
    bf16x8 aq[RB][3];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int term = 0; term < 3; ++term)
        aq[rb][term] = as_bf16x8(slot[(hb * 3 + term) * BM + rb * 32 + rr]);
    mfma_split6<RB, 1>(aq, bq, lo, hi);
    if constexpr ((K + 1) % (kSubChunk / 16) == 0) flush_hi_fp64(sumd, hi);
    if constexpr ((K + 1) % PERIOD == 0) barrier();
  };
  static_assert(24 % (kSubChunk / 16) == 0 && 24 % NSL == 0 && 24 % PERIOD == 0 && 24 % 3 == 0,
                "the unrolled steps repeat every slot, set and flush pattern");

  // prologue: M stages 0 .. 3 in their slots, stages 4 .. 6 in registers,
  // screen stages 0 .. 3 in registers
  for (int st = 0; st < AHEAD; ++st)
    ringA[st][tid] = *(const uint4*)(srcA + (size_t)min(st, nst - 1) * advA);
  load_a(std::integral_constant<int, 0>{}, min(AHEAD, nst - 1));
  load_a(std::integral_constant<int, 1>{}, min(AHEAD + 1, nst - 1));
  load_a(std::integral_constant<int, 2>{}, min(AHEAD + 2, nst - 1));
  load_b(std::integral_constant<int, 0>{}, 0);
  load_b(std::integral_constant<int, 1>{}, 1);
  load_b(std::integral_constant<int, 2>{}, 2);
  load_b(std::integral_constant<int, 3>{}, 3);
  barrier();
  int s0 = 0;
  for (; s0 + 24 <= nst; s0 += 24)
    unroll_steps<24>([&](auto kc) __attribute__((always_inline)) {
      step(kc, s0 + decltype(kc)::value);
    });
  unroll_steps<23>([&](auto kc) __attribute__((always_inline)) {
    if (s0 + decltype(kc)::value < nst) step(kc, s0 + decltype(kc)::value);
  });

  const int gcol = t.col0 + col;
  const int j = gcol >> 1;
  const int cmp = gcol & 1;
  if (j >= P || j >= t.pad[0]) return;
  const int nr = nrhoSorted[j];
  double* dst = part + ((size_t)t.kc * lineTotal + lineOffSorted[j]) * 2 + cmp;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    if (rb >= t.rbN) break;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = t.row0 + rb * 32 + 8 * (r >> 2) + 4 * hb + (r & 3);
      if (row < nr) dst[(size_t)row * 2] = sumd[rb][r] + (double)lo[rb][r];
    }
  }
}

// --------------------------------------------------------------------------
// FP32 contraction through the same FP32 ring: v_mfma_f32_32x32x2f32, FP32
// sums over kSubChunk nodes added to FP64 running sums.
// --------------------------------------------------------------------------
template <int WR, int WC, int RBW, int CBW, int NS>
__global__ __launch_bounds__(64 * WR * WC) void k_contract_f32_ringf(
    const Tile* __restrict__ tiles, int NrPad, int kchunk, int P, int lineTotal,
    const float* __restrict__ M32, const float* __restrict__ B32,
    const int32_t* __restrict__ nrhoSorted, const int32_t* __restrict__ lineOffSorted,
    double* __restrict__ part) {
  constexpr int BM = 32 * RBW * WR;
  constexpr int BN = 32 * CBW * WC;
  constexpr int NT = 64 * WR * WC;          // threads
  constexpr int AU = BM * 4;                // 16-byte quarters of M per stage
  constexpr int SU = AU + BN * 4;           // quarters per stage
  // LF load rounds of every wave, then one more by the first RW waves
  constexpr int LF = SU / NT;
  constexpr int RW = (SU - LF * NT) / 64;
  constexpr int LW = LF + (RW > 0 ? 1 : 0);
  constexpr int SLOT = SU;
  static_assert(SU % 64 == 0, "whole waves of quarters");
  static_assert(LW * (NS - 2) < 64, "too many loads in flight for vmcnt");
  static_assert(NS == 4 || NS == 8, "ring depth");
  __shared__ float4 ring0[SLOT];
  __shared__ float4 ring1[SLOT];
  __shared__ float4 ring2[SLOT];
  __shared__ float4 ring3[SLOT];
  __shared__ float4 ring4[NS > 4 ? SLOT : 1];
  __shared__ float4 ring5[NS > 4 ? SLOT : 1];
  __shared__ float4 ring6[NS > 4 ? SLOT : 1];
  __shared__ float4 ring7[NS > 4 ? SLOT : 1];

  const Tile t = tiles[blockIdx.x];
  if (t.row0 < 0) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave / WC;
  const int wc = wave - wr * WC;
  const int hb = lane >> 5;
  const int rr = lane & 31;

  // source of slot position u = 256 l + tid: position 4 r + q' holds quarter
  // q' ^ ((r / 4) % 4) of row (or column) r; stage s adds 16 nodes
  const float* src[LW];
#pragma unroll
  for (int l = 0; l < LW; ++l) {
    int u = NT * l + tid;
    if (u >= SU) u = 0;  // waves past the last partial round: never issued
    if (u < AU) {
      const int r = u >> 2;
      const int qd = (u & 3) ^ ((r >> 2) & 3);
      src[l] = M32 + (size_t)(t.row0 + r) * NrPad + t.k0 + 4 * qd;
    } else {
      const int c = (u - AU) >> 2;
      const int qd = ((u - AU) & 3) ^ ((c >> 2) & 3);
      src[l] = B32 + (size_t)(t.col0 + c) * NrPad + t.k0 + 4 * qd;
    }
  }
  const int nst = kchunk / 16;  // a multiple of 16

  double accd[RBW * CBW][16];
  f32x16 hi[RBW * CBW];
#pragma unroll
  for (int b = 0; b < RBW * CBW; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      accd[b][r] = 0.0;
      hi[b][r] = 0.f;
    }
  const int rbBase = wr * RBW;

  auto slot_of = [&](auto kc) -> float4* {
    constexpr int K = decltype(kc)::value;
    if constexpr (K == 0) return ring0;
    else if constexpr (K == 1) return ring1;
    else if constexpr (K == 2) return ring2;
    else if constexpr (K == 3) return ring3;
    else if constexpr (K == 4) return ring4;
    else if constexpr (K == 5) return ring5;
    else if constexpr (K == 6) return ring6;
    else return ring7;
  };
  auto issue = [&](auto kc, int stage) {
    float4* slot = slot_of(kc);
#pragma unroll
    for (int l = 0; l < LW; ++l)
      if (l < LF || wave < RW)  // wave-uniform
        __builtin_amdgcn_global_load_lds((const void*)(src[l] + (size_t)stage * 16),
                                         (__attribute__((address_space(3))) void*)(slot + NT * l +
                                                                                   64 * wave),
                                         16, 0, 0);
  };
  auto barrier = [&]() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };
  // the 8 nodes hb*8 .. hb*8 + 7 of row (or column) r of a slot region
  auto fragment = [&](const float4* region, int r, float4& lo4, float4& hi4) {
    const int sw = (r >> 2) & 3;
    lo4 = region[4 * r + ((2 * hb) ^ sw)];
    hi4 = region[4 * r + ((2 * hb + 1) ^ sw)];
  };
  auto step = [&](auto kc, int s) {
    constexpr int K = decltype(kc)::value;
    constexpr int KN = (K + NS - 1) % NS;
    if (s + NS - 2 < nst) {
      if (RW == 0 || wave < RW)
        wait_vmcnt<LW * (NS - 2)>();
      else
        wait_vmcnt<LF * (NS - 2)>();
    } else {
      wait_vmcnt<0>();
    }
    barrier();
    if (s + NS - 1 < nst) issue(std::integral_constant<int, KN>{}, s + NS - 1);
    const float4* slot = slot_of(kc);
    float bq[CBW][8];
#pragma unroll
    for (int cb = 0; cb < CBW; ++cb) {
      float4 a, b;
      fragment(slot + AU, wc * 32 * CBW + cb * 32 + rr, a, b);
      bq[cb][0] = a.x; bq[cb][1] = a.y; bq[cb][2] = a.z; bq[cb][3] = a.w;
      bq[cb][4] = b.x; bq[cb][5] = b.y; bq[cb][6] = b.z; bq[cb][7] = b.w;
    }
    float aq[RBW][8];
#pragma unroll
    for (int rb = 0; rb < RBW; ++rb) {
      float4 a, b;
      fragment(slot, (rbBase + rb) * 32 + rr, a, b);
      aq[rb][0] = a.x; aq[rb][1] = a.y; aq[rb][2] = a.z; aq[rb][3] = a.w;
      aq[rb][4] = b.x; aq[rb][5] = b.y; aq[rb][6] = b.z; aq[rb][7] = b.w;
    }
    // K-step kk pairs node kk (lanes 0-31) with node 8 + kk (lanes 32-63), in
    // A and B alike, so the 8 steps cover the stage's 16 nodes
#pragma unroll
    for (int kk = 0; kk < 8; ++kk)
#pragma unroll
      for (int rb = 0; rb < RBW; ++rb)
#pragma unroll
        for (int cb = 0; cb < CBW; ++cb)
          hi[rb * CBW + cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(aq[rb][kk], bq[cb][kk],
                                                                   hi[rb * CBW + cb], 0, 0, 0);
    if (((s + 1) * 16) % kSubChunk == 0) {
#pragma unroll
      for (int b = 0; b < RBW * CBW; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          accd[b][r] += (double)hi[b][r];
          hi[b][r] = 0.f;
        }
    }
  };

  issue(std::integral_constant<int, 0>{}, 0);
  issue(std::integral_constant<int, 1>{}, 1);
  issue(std::integral_constant<int, 2>{}, 2);
  if constexpr (NS == 8) {
    issue(std::integral_constant<int, 3>{}, 3);
    issue(std::integral_constant<int, 4>{}, 4);
    issue(std::integral_constant<int, 5>{}, 5);
    issue(std::integral_constant<int, 6>{}, 6);
  }
  for (int s0 = 0; s0 < nst; s0 += NS) {
    step(std::integral_constant<int, 0>{}, s0);
    step(std::integral_constant<int, 1>{}, s0 + 1);
    step(std::integral_constant<int, 2>{}, s0 + 2);
    step(std::integral_constant<int, 3>{}, s0 + 3);
    if constexpr (NS == 8) {
      step(std::integral_constant<int, 4>{}, s0 + 4);
      step(std::integral_constant<int, 5>{}, s0 + 5);
      step(std::integral_constant<int, 6>{}, s0 + 6);
      step(std::integral_constant<int, 7>{}, s0 + 7);
    }
  }

#pragma unroll
  for (int cb = 0; cb < CBW; ++cb) {
    const int col = t.col0 + wc * 32 * CBW + cb * 32 + rr;
    const int j = col >> 1;
    const int comp = col & 1;
    if (j >= P || j >= t.pad[0]) continue;
    const int nr = nrhoSorted[j];
    double* dst = part + ((size_t)t.kc * lineTotal + lineOffSorted[j]) * 2 + comp;
#pragma unroll
    for (int rb = 0; rb < RBW; ++rb) {
      if (rbBase + rb >= t.rbN) break;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = t.row0 + (rbBase + rb) * 32 + 8 * (r >> 2) + 4 * hb + (r & 3);
        if (row < nr) dst[(size_t)row * 2] = accd[rb * CBW + cb][r];
      }
    }
  }
}

// --------------------------------------------------------------------------
// Spline coefficients (section 4.3.2).  One wave per sorted plane.  The
// second derivatives m of the interpolating cubic spline with s'(0) = 0 and
// s''(n-1) = 0 solve T m = d with rows
//   2 m_0 + m_1 = 6 (y_1 - y_0),
//   m_{k-1} + 4 m_k + m_{k+1} = 6 (y_{k-1} - 2 y_k + y_{k+1}),  m_{n-1} = 0.
// Thomas elimination: d'_0 = d_0 / 2, d'_k = (d_k - d'_{k-1}) c'_k with the
// data-independent c'_0 = 1/2, c'_k = 1 / (4 - c'_{k-1}) (table from the
// plan), then m_k = d'_k - c'_k m_{k+1}.  Both recurrences damp an error in
// their start value by c'_k ~ 0.268 per step, so each lane runs them over
// its own segment of nodes from kSplineWarm nodes outside it with a zero
// start value (exact at the ends of the line, where the true start values
// are known) and no lane waits for another.  The partial sums of the
// contraction's K-chunks are combined here in FP64.
// Output per interval k: power-form coefficients c0..c3 of re and im,
//   s(k + u) = c0 + u (c1 + u (c2 + u c3)),  u in [0, 1).
// (A 16-byte-per-node layout halves the resample's LDS, but measured 3-4%
// slower on the batch workload: the higher occupancy did not help the
// write stream.)
// --------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_spline(int j0, int nkc, int lineTotal, int interp,
                                               const int32_t* __restrict__ nrhoSorted,
                                               const int32_t* __restrict__ lineOffSorted,
                                               const double* __restrict__ cprime,
                                               const double* __restrict__ part,
                                               float4* __restrict__ coef, double frac2,
                                               int qos, int32_t* __restrict__ hTrunc,
                                               const int32_t* __restrict__ perm,
                                               int32_t* __restrict__ status) {
  extern __shared__ double2 smem[];
  // c'_k for k < 64; the recurrence reaches its FP64 fixed point by k = 15,
  // so c'_k = c'_63 for every k >= 63
  __shared__ double cpL[64];
  const int j = j0 + blockIdx.x;
  const int lane = threadIdx.x;
  const int n = nrhoSorted[j];
  const int off = lineOffSorted[j];
  double2* y = smem;           // [n] radial line
  double2* dp = smem + n;      // [n] eliminated right-hand side d'
  double2* m = smem + 2 * n;   // [n] second derivatives
  cpL[lane] = cprime[min(lane, n - 1)];
  auto cp = [&](int k) { return cpL[min(k, 63)]; };

  // the K-chunk partial sums, added in chunk order, eight nodes per lane in
  // flight (loads past the line re-read its last node and are dropped)
  const double2* partL = (const double2*)part + off;
  bool finite = true;
  for (int k0 = lane; k0 < n; k0 += 64 * 8) {
    double2 acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = make_double2(0.0, 0.0);
    for (int c = 0; c < nkc; ++c) {
      double2 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = partL[(size_t)c * lineTotal + min(k0 + 64 * u, n - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        acc[u].x += v[u].x;
        acc[u].y += v[u].y;
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k0 + 64 * u < n) {
        y[k0 + 64 * u] = acc[u];
        finite = finite && isfinite(acc[u].x) && isfinite(acc[u].y);
      }
  }
  // a non-finite line value (from a non-finite taper sample or w) sets the
  // plan's status word; the line's cache is then unspecified
  if (__any(!finite) && lane == 0) {
    atomicOr(&status[0], kStatusNonFinite);
    atomicMin(&status[1], perm[j]);
  }
  __syncthreads();

  if (hTrunc) {
    // truncation (section 3.1): last node with |y_k|^2 >= frac^2 max |y|^2;
    // half-width ceil(k* / (q os)), at most the planned (n - 4) / (q os)
    double mx = 0.0;
    for (int k = lane; k < n; k += 64) mx = fmax(mx, y[k].x * y[k].x + y[k].y * y[k].y);
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    int last = 0;
    for (int k = lane; k < n; k += 64)
      if (y[k].x * y[k].x + y[k].y * y[k].y >= frac2 * mx) last = max(last, k);
    for (int o = 32; o > 0; o >>= 1) last = max(last, __shfl_xor(last, o));
    if (lane == 0) hTrunc[j] = min((last + qos - 1) / qos, (n - 4) / qos);
  }

  const int L = (n + 63) / 64;
  const int s = min(lane * L, n);
  const int e = min(s + L, n);

  if (interp == 1) {
    // forward elimination over rows 0 .. n-2 (row n-1 gives d' = 0)
    {
      const int start = max(0, s - kSplineWarm);
      double2 prev = make_double2(0.0, 0.0);
#pragma unroll 4
      for (int k = start; k < e; ++k) {
        double2 v;
        if (k == n - 1) {
          v = make_double2(0.0, 0.0);
        } else if (k == 0) {
          v.x = 6.0 * (y[1].x - y[0].x) * cp(0);
          v.y = 6.0 * (y[1].y - y[0].y) * cp(0);
        } else {
          const double dx = 6.0 * (y[k - 1].x - 2.0 * y[k].x + y[k + 1].x);
          const double dy = 6.0 * (y[k - 1].y - 2.0 * y[k].y + y[k + 1].y);
          v.x = (dx - prev.x) * cp(k);
          v.y = (dy - prev.y) * cp(k);
        }
        prev = v;
        if (k >= s) dp[k] = v;
      }
    }
    __syncthreads();
    // back substitution: m_{n-1} = 0, m_k = d'_k - c'_k m_{k+1}
    {
      const int top = min(n - 1, e - 1 + kSplineWarm);
      double2 next = make_double2(0.0, 0.0);  // m_{top + 1}; exact when top == n-1
#pragma unroll 4
      for (int k = top; k >= s; --k) {
        double2 v;
        if (k == n - 1) {
          v = make_double2(0.0, 0.0);
        } else {
          v.x = dp[k].x - cp(k) * next.x;
          v.y = dp[k].y - cp(k) * next.y;
        }
        next = v;
        if (k < e) m[k] = v;
      }
    }
    __syncthreads();
  }

  for (int k = s; k < e; ++k) {
    float4 cr, ci;
    if (k <= n - 2) {
      const double2 y0 = y[k], y1 = y[k + 1];
      if (interp == 1) {
        // thirds and sixths as products with the rounded reciprocals (within
        // an FP64 ulp of the quotients, far below the FP32 the coefficients
        // are stored in; an FP64 division costs about ten instructions)
        const double2 m0 = m[k], m1 = m[k + 1];
        const double r3 = 1.0 / 3.0, r6 = 1.0 / 6.0;
        cr = make_float4((float)y0.x, (float)(y1.x - y0.x - m0.x * r3 - m1.x * r6),
                         (float)(0.5 * m0.x), (float)((m1.x - m0.x) * r6));
        ci = make_float4((float)y0.y, (float)(y1.y - y0.y - m0.y * r3 - m1.y * r6),
                         (float)(0.5 * m0.y), (float)((m1.y - m0.y) * r6));
      } else {
        cr = make_float4((float)y0.x, (float)(y1.x - y0.x), 0.f, 0.f);
        ci = make_float4((float)y0.y, (float)(y1.y - y0.y), 0.f, 0.f);
      }
    } else {
      cr = make_float4((float)y[k].x, 0.f, 0.f, 0.f);
      ci = make_float4((float)y[k].y, 0.f, 0.f, 0.f);
    }
    coef[(size_t)(off + k) * 2] = cr;
    coef[(size_t)(off + k) * 2 + 1] = ci;
  }
}

// Radial lines in caller order (complex128), K-chunk partial sums combined;
// a mirrored plane gets the conjugate of its source's line.
__global__ void k_lines_out(int Pall, int nkc, int lineTotal, const PlaneInfo* __restrict__ planes,
                            const double* __restrict__ part, double2* __restrict__ lines) {
  const int p = blockIdx.y;
  if (p >= Pall) return;
  const PlaneInfo pi = planes[p];
  const double sgn = pi.conj ? -1.0 : 1.0;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < pi.nrho; k += gridDim.x * blockDim.x) {
    double re = 0.0, im = 0.0;
    for (int c = 0; c < nkc; ++c) {
      const double2 v = ((const double2*)part)[(size_t)c * lineTotal + pi.line_off + k];
      re += v.x;
      im += v.y;
    }
    lines[pi.line_off_caller + k] = make_double2(re, sgn * im);
  }
}

// ==========================================================================
// Adjoint (gradient of a real loss of the kernel cache).  The paper has no
// gradient; these kernels apply the transposes of the forward steps in
// reverse order, in FP64, with every reduction in a fixed order (no atomics),
// so the result is bit-reproducible.
// ==========================================================================

// Resample transpose, part 1 (every plane, caller order, moments stored in the
// caller-order line layout; a mirrored plane's cache is the conjugate of
// its source's, so its gradient enters conjugated): for interval k of plane
// p the moments
//   g_j[k] = sum over cache samples e with interval(e) = k of u(e)^j G(e),
// j = 0..3 (the gradients of the power-form coefficients c0..c3).
//
// One thread per sample, over the resample units (coalesced reads): the
// sample's interval and fraction come from the forward's own radial_pos, so
// this is exactly the transpose of what the forward evaluated.  Each product
// u^j G is formed in FP64 and added as a 64-bit fixed-point integer, first
// into the workgroup's LDS bins and then into the global bins: integer sums
// do not depend on the order of the additions, so the result is
// bit-reproducible without a fixed reduction order.  The fixed-point scale of
// plane p is 2^E_p with E_p = 60 - eN - e_p, where max |G| < 2^e_p (a
// pre-pass) and 2^eN bounds the samples of one interval: every sum stays
// below 2^60 and the quantum is at most 2^(eN - 59) max |G| (about 1e-13 of
// it for eN = 16), well inside what FP64 accumulation of the same products
// keeps.  A plane whose G holds a non-finite value gets NaN moments.
constexpr int kMomThreads = 256;

__device__ __forceinline__ int moment_exponent(uint32_t amaxBits, int eN) {
  int e = 0;
  (void)frexpf(__uint_as_float(amaxBits), &e);  // 0 for max |G| = 0
  return 60 - eN - e;
}

// Zeroes the fixed-point bins [n8] and the per-plane maxima [P].
__global__ void k_grad_clear(int64_t n8, unsigned long long* __restrict__ fx, int P,
                             uint32_t* __restrict__ amax) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = i; j < n8; j += stride) fx[j] = 0ull;
  for (int64_t j = i; j < P; j += stride) amax[j] = 0u;
}

// Per-plane max |Re G|, |Im G| as FP32 bits (a non-finite value counts as
// +inf); max is order independent.
__global__ __launch_bounds__(256) void k_grad_absmax(const ResampleUnit* __restrict__ units,
                                                     const PlaneInfo* __restrict__ planes,
                                                     const float2* __restrict__ g,
                                                     uint32_t* __restrict__ amax) {
  __shared__ float red[4];
  const ResampleUnit u = units[blockIdx.x];
  const float2* gp = g + planes[u.p].out_off;
  float m = 0.f;
  auto take = [&](float2 v) {
    const float a = fmaxf(fabsf(v.x), fabsf(v.y));
    m = fmaxf(m, (isfinite(v.x) && isfinite(v.y)) ? a : __builtin_inff());
  };
  int e = u.e0 + (int)threadIdx.x;
  for (; e + 7 * 256 < u.e1; e += 8 * 256) {
    float2 v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = gp[e + i * 256];
#pragma unroll
    for (int i = 0; i < 8; ++i) take(v[i]);
  }
  for (; e < u.e1; e += 256) take(gp[e]);
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    atomicMax(amax + u.p, __float_as_uint(m));
  }
}

// FP64 value (|x| < 2^62) rounded to the nearest 64-bit integer.
__device__ __forceinline__ unsigned long long fixed_round(double x) {
  const double r = __builtin_rint(x);
  const double hi = __builtin_floor(r * 0x1p-32);
  const double lo = __builtin_fma(-hi, 0x1p32, r);  // exact, in [0, 2^32)
  return ((unsigned long long)(long long)(int)hi << 32) + (unsigned long long)(uint32_t)lo;
}

__global__ __launch_bounds__(kMomThreads) void k_resample_T(
    const ResampleUnit* __restrict__ units, const PlaneInfo* __restrict__ planes, int os,
    float invOs, float q, int eN, const uint32_t* __restrict__ amax,
    const float2* __restrict__ g, unsigned long long* __restrict__ fx) {
  extern __shared__ unsigned long long bins[];  // [8][nrho]: consecutive k in consecutive banks
  const ResampleUnit un = units[blockIdx.x];
  const PlaneInfo pi = planes[un.p];
  const int n = pi.nrho;
  const int nmax = n - 2;
  for (int i = threadIdx.x; i < n * 8; i += kMomThreads) bins[i] = 0ull;
  const uint32_t am = amax[un.p];
  if (!(__uint_as_float(am) <= 3.4028235e38f)) return;  // uniform: NaN moments
  const double sc = __builtin_ldexp(1.0, moment_exponent(am, eN));
  const double ysc = pi.conj ? -sc : sc;
  const float2* gp = g + pi.out_off;
  const int S = pi.S, h = pi.h;
  __syncthreads();
  const int lim = pi.lim;
  auto take = [&](int e, int X, int Y) {
    const int d2 = X * X + Y * Y;
    if (d2 > lim) return;
    int k;
    float uu;
    radial_pos(d2, q, nmax, k, uu);
    const float2 gv = gp[e];
    const double gx = sc * gv.x, gy = ysc * gv.y;
    const double u1 = uu, u2 = u1 * u1, u3 = u2 * u1;
    unsigned long long* bk = bins + k;
    atomicAdd(bk + 0 * n, fixed_round(gx));
    atomicAdd(bk + 1 * n, fixed_round(gy));
    atomicAdd(bk + 2 * n, fixed_round(u1 * gx));
    atomicAdd(bk + 3 * n, fixed_round(u1 * gy));
    atomicAdd(bk + 4 * n, fixed_round(u2 * gx));
    atomicAdd(bk + 5 * n, fixed_round(u2 * gy));
    atomicAdd(bk + 6 * n, fixed_round(u3 * gx));
    atomicAdd(bk + 7 * n, fixed_round(u3 * gy));
  };
  if (S >= 64) {
    // Wave w takes the 64-sample chunks w, w + 4, ... of the unit (units
    // start at multiples of 256); a chunk's first sample is decoded once
    // and advanced by 256 samples a step, and a chunk crosses at most one
    // row boundary.
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int e = un.e0 + 64 * wave;
    int rem;
    const int R = div_small(e, S, pi.invS, rem);
    int a0 = rem;
    const int F = div_small(R, S, pi.invS, rem);
    int b0 = rem;
    int fv0 = div_small(F, os, invOs, rem);
    int fu0 = rem;
    const int stepA = 256 % S;
    const int stepR = 256 / S;
    for (; e < un.e1; e += 256) {
      if (e + lane < un.e1) {
        int a = a0 + lane, b = b0, fu = fu0, fv = fv0;
        if (a >= S) {
          a -= S;
          if (++b == S) {
            b = 0;
            if (++fu == os) {
              fu = 0;
              ++fv;
            }
          }
        }
        take(e + lane, os * (a - h) - fu, os * (b - h) - fv);
      }
      a0 += stepA;
      int c = stepR;
      if (a0 >= S) {
        a0 -= S;
        ++c;
      }
      b0 += c;
      if (b0 >= S) {
        b0 -= S;
        if (++fu0 == os) {
          fu0 = 0;
          ++fv0;
        }
      }
    }
  } else {
    for (int e = un.e0 + (int)threadIdx.x; e < un.e1; e += kMomThreads) {
      int a, b, fu;
      const int R = div_small(e, S, pi.invS, a);
      const int F = div_small(R, S, pi.invS, b);
      const int fv = div_small(F, os, invOs, fu);
      take(e, os * (a - h) - fu, os * (b - h) - fv);
    }
  }
  __syncthreads();
  unsigned long long* dst = fx + (size_t)pi.line_off_caller * 8;
  for (int i = threadIdx.x; i < n * 8; i += kMomThreads) {
    const int k = i >> 3;
    const unsigned long long v = bins[(i & 7) * n + k];
    if (v) atomicAdd(dst + i, v);
  }
}

// Fixed-point bins -> FP64 moments [lineTotalAll][4] (caller order).
__global__ void k_mom_convert(const PlaneInfo* __restrict__ planes, int eN,
                              const uint32_t* __restrict__ amax,
                              const unsigned long long* __restrict__ fx,
                              double2* __restrict__ mom) {
  const int p = blockIdx.y;
  const PlaneInfo pi = planes[p];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= pi.nrho) return;
  const uint32_t am = amax[p];
  const bool ok = __uint_as_float(am) <= 3.4028235e38f;
  const double inv = __builtin_ldexp(1.0, -moment_exponent(am, eN));
  const size_t L = (size_t)pi.line_off_caller + k;
  for (int j = 0; j < 4; ++j) {
    const double re = (double)(long long)fx[L * 8 + 2 * j] * inv;
    const double im = (double)(long long)fx[L * 8 + 2 * j + 1] * inv;
    mom[L * 4 + j] = ok ? make_double2(re, im) : make_double2(__builtin_nan(""), __builtin_nan(""));
  }
}

// Resample transpose, part 2: coefficient moments -> gradient of the radial
// line.  c0 = y_k, c1 = y_{k+1} - y_k - m_k/3 - m_{k+1}/6, c2 = m_k/2,
// c3 = (m_{k+1} - m_k)/6 give dL/dy and dL/dm; the second derivatives are
// m = T^-1 D y, so dL/dy += D^T T^-T dL/dm.  T^T has the rows [2 1],
// [1 4 1] ... [1 4 0], [1 1], so its Thomas factors are the forward spline's
// c'_k up to row n - 3, c'_{n-2} = 0, and a last pivot of 1.  One wave per
// sorted plane, the line in LDS; like the forward spline, every lane runs the
// elimination and the back substitution over its own segment from
// kSplineWarm nodes outside it with a zero start value (damped by c'_k ~
// 0.27 per node), exact at the two ends of the line.  Mirrored planes add
// their moments to their source's, in a fixed order.
__global__ __launch_bounds__(64) void k_spline_T(int j0, int interp,
                                                 const int32_t* __restrict__ perm,
                                                 const int32_t* __restrict__ nrhoSorted,
                                                 const int32_t* __restrict__ lineOffSorted,
                                                 const int32_t* __restrict__ lineOffCaller,
                                                 const int32_t* __restrict__ mirStart,
                                                 const int32_t* __restrict__ mirList,
                                                 const double* __restrict__ cprime,
                                                 const double2* __restrict__ mom,
                                                 double2* __restrict__ gy) {
  extern __shared__ double2 smT[];
  const int j = j0 + blockIdx.x;
  const int lane = threadIdx.x;
  const int n = nrhoSorted[j];
  const double2* M = mom + (size_t)lineOffCaller[perm[j]] * 4;
  const int mi0 = mirStart[j], mi1 = mirStart[j + 1];
  double2* y = smT;          // [n] dL/dy
  double2* m = smT + n;      // [n] dL/dm, then the eliminated d'
  double2* z = smT + 2 * n;  // [n] T^-T dL/dm
  // moments of interval k, mirrored planes added in a fixed order
  auto moments = [&](int k, double2 (&g)[4]) {
#pragma unroll
    for (int t = 0; t < 4; ++t) g[t] = M[4 * k + t];
    for (int mi = mi0; mi < mi1; ++mi) {
      const double2* Mm = mom + (size_t)lineOffCaller[mirList[mi]] * 4;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        g[t].x += Mm[4 * k + t].x;
        g[t].y += Mm[4 * k + t].y;
      }
    }
  };
  for (int k = lane; k < n; k += 64) {
    double2 yk = make_double2(0.0, 0.0), mk = make_double2(0.0, 0.0);
    double2 g[4];
    if (k >= 1) {  // from interval k - 1 (every interval below n - 1 has a cubic)
      moments(k - 1, g);
      yk.x += g[1].x;
      yk.y += g[1].y;
      if (interp == 1) {
        mk.x += -g[1].x / 6.0 + g[3].x / 6.0;
        mk.y += -g[1].y / 6.0 + g[3].y / 6.0;
      }
    }
    moments(k, g);
    if (k == n - 1) {  // the last node's interval is the constant y_{n-1}
      yk.x += g[0].x;
      yk.y += g[0].y;
    } else {
      yk.x += g[0].x - g[1].x;
      yk.y += g[0].y - g[1].y;
      if (interp == 1) {
        mk.x += -g[1].x / 3.0 + 0.5 * g[2].x - g[3].x / 6.0;
        mk.y += -g[1].y / 3.0 + 0.5 * g[2].y - g[3].y / 6.0;
      }
    }
    y[k] = yk;
    m[k] = mk;
  }
  __syncthreads();
  if (interp == 1) {
    const int L = (n + 63) / 64;
    const int s0 = min(lane * L, n);
    const int e0 = min(s0 + L, n);
    // elimination, rows 0 .. n-1, over [start, e0) with a zero start value
    {
      const int start = max(0, s0 - kSplineWarm);
      double2 prev = make_double2(0.0, 0.0);
      for (int k = start; k < e0; ++k) {
        double2 v;
        if (k == 0) {
          v.x = 0.5 * m[0].x;
          v.y = 0.5 * m[0].y;
        } else if (k == n - 1) {
          v.x = m[k].x - prev.x;
          v.y = m[k].y - prev.y;
        } else {
          v.x = (m[k].x - prev.x) * cprime[k];
          v.y = (m[k].y - prev.y) * cprime[k];
        }
        prev = v;
        if (k >= s0) z[k] = v;  // z holds d' until the back substitution
      }
    }
    __syncthreads();
    for (int k = s0; k < e0; ++k) m[k] = z[k];  // d'
    __syncthreads();
    // back substitution z_k = d'_k - c'_k z_{k+1} (c'_{n-2} = 0, z_{n-1} = d'_{n-1})
    {
      const int top = min(n - 1, e0 - 1 + kSplineWarm);
      double2 next = make_double2(0.0, 0.0);
      for (int k = top; k >= s0; --k) {
        double2 v = m[k];
        if (k <= n - 3) {
          v.x -= cprime[k] * next.x;
          v.y -= cprime[k] * next.y;
        }
        next = v;
        if (k < e0) z[k] = v;
      }
    }
    __syncthreads();
    // y += D^T z: D rows 0: [-6, 6]; k = 1..n-2: [6, -12, 6]; n-1: 0
    for (int i = lane; i < n; i += 64) {
      double ax = 0.0, ay = 0.0;
      if (i >= 1 && i - 1 <= n - 2) {
        ax += 6.0 * z[i - 1].x;
        ay += 6.0 * z[i - 1].y;
      }
      if (i <= n - 2) {
        const double dd = i == 0 ? -6.0 : -12.0;
        ax += dd * z[i].x;
        ay += dd * z[i].y;
      }
      if (i + 1 >= 1 && i + 1 <= n - 2) {
        ax += 6.0 * z[i + 1].x;
        ay += 6.0 * z[i + 1].y;
      }
      y[i].x += ax;
      y[i].y += ay;
    }
    __syncthreads();
  }
  double2* out = gy + lineOffSorted[j];
  for (int k = lane; k < n; k += 64) out[k] = y[k];
}

// Transposed Hankel contraction and screen backward:
//   G_s[i] = sum_k M[k, i] gy_j[k],  u = G_s exp(-j theta_i),
//   ure[j][i] = Re u,  wterm[j][i] = 2 pi phi_i tau_i Im u,
// theta = 2 pi w phi with the phase reduced modulo 1 in FP64.
__global__ __launch_bounds__(256) void k_contract_T(
    int Nr, int NrPad, const int32_t* __restrict__ perm, const int32_t* __restrict__ nrhoSorted,
    const int32_t* __restrict__ lineOffSorted, const float* __restrict__ M32,
    const double* __restrict__ phi, const float* __restrict__ taper,
    const double* __restrict__ w, const double2* __restrict__ gy, double* __restrict__ ure,
    double* __restrict__ wterm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= Nr) return;
  const int n = nrhoSorted[j];
  const double2* y = gy + lineOffSorted[j];
  const float* mcol = M32 + i;
  double gr = 0.0, gi = 0.0;
  int k = 0;
  // eight loads in flight per step; the sums still run over k in order
  for (; k + 8 <= n; k += 8) {
    float mk[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) mk[t] = mcol[(size_t)(k + t) * NrPad];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const double2 v = y[k + t];
      gr += (double)mk[t] * v.x;
      gi += (double)mk[t] * v.y;
    }
  }
  for (; k < n; ++k) {
    const double mk = (double)mcol[(size_t)k * NrPad];
    const double2 v = y[k];
    gr += mk * v.x;
    gi += mk * v.y;
  }
  double t = w[perm[j]] * phi[i];
  t -= rint(t);
  double sn, cs;
  sincospi(2.0 * t, &sn, &cs);
  const double ur = gr * cs + gi * sn;
  const double ui = gi * cs - gr * sn;
  ure[(size_t)j * NrPad + i] = ur;
  wterm[(size_t)j * NrPad + i] = kTwoPi * phi[i] * (double)taper[i] * ui;
}

// dL/dtau_i = sum over planes (sorted order) of Re u: thread (x, y) of a
// block adds the planes y, y + 8, ... of node i in order, and the eight
// partial sums are added in y order (a fixed order: bit-reproducible).
__global__ __launch_bounds__(256) void k_grad_taper(int P, int Nr, int NrPad,
                                                    const double* __restrict__ ure,
                                                    float* __restrict__ gtau) {
  __shared__ double part[8][32];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int i = blockIdx.x * 32 + tx;
  double acc = 0.0;
  if (i < Nr)
    for (int j = ty; j < P; j += 8) acc += ure[(size_t)j * NrPad + i];
  part[ty][tx] = acc;
  __syncthreads();
  if (ty == 0 && i < Nr) {
    double t = part[0][tx];
    for (int g = 1; g < 8; ++g) t += part[g][tx];
    gtau[i] = (float)t;
  }
}

// dL/dw of mirrored planes is folded into their sources.
__global__ void k_grad_w_mirrored(int n, const int32_t* __restrict__ mirList,
                                  double* __restrict__ gw) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) gw[mirList[i]] = 0.0;
}

// dL/dw_p = sum_i wterm[j][i]: per-thread strided sums, then a fixed tree.
__global__ __launch_bounds__(256) void k_grad_w(int Nr, int NrPad,
                                                const int32_t* __restrict__ perm,
                                                const double* __restrict__ wterm,
                                                double* __restrict__ gw) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < Nr; i += 256) acc += wterm[(size_t)j * NrPad + i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int stride = 128; stride > 0; stride >>= 1) {
    if ((int)threadIdx.x < stride) red[threadIdx.x] += red[threadIdx.x + stride];
    __syncthreads();
  }
  if (threadIdx.x == 0) gw[perm[j]] = red[0];
}

// --------------------------------------------------------------------------
// Projection-slice engine (section 4.3.1, Algorithm 2): the radial line of a
// plane from its IConv-kernel sampled on an N x N workspace (pixel
// l = (x - N/2) FOV/N, zero outside the open disc r < r_max, taper linear
// in r between its midpoint samples), projected onto the l axis and
// transformed with zero padding by q os:
//   p(l_i) = dl sum_j s(l_i, m_j),  K(rho_k) = dl sum_i p(l_i) e^{-j 2 pi rho_k l_i}.
// The sampled screen is even in both axes (the row and column at -N/2 lie
// outside the disc), so with c = N/2 and offsets i, j in [0, c):
//   p_i = dl (s(i, 0) + 2 sum_{j>0} s(i, j)),
//   K_k = dl (p_0 + 2 sum_{i>0} p_i cos(2 pi k i / (q os N))).
// Inside the disc iff i^2 + j^2 < c^2 (exact in integers).  FP64 throughout;
// one workgroup per sorted plane; the cosine table comes from the plan,
// sampled at stride Lmax / L for this plane's L = q os N.
// --------------------------------------------------------------------------
__device__ __forceinline__ double taper_at(double r, double dr, int Nr,
                                           const float* __restrict__ taper) {
  const double t = r / dr - 0.5;
  if (t <= 0.0) return (double)taper[0];
  const int i0 = (int)t;
  if (i0 >= Nr - 1) return (double)taper[Nr - 1];
  const double a = (double)taper[i0];
  return a + (t - (double)i0) * ((double)taper[i0 + 1] - a);
}

constexpr int kPsThreads = 256;

__global__ __launch_bounds__(kPsThreads) void k_ps_lines(
    int j0, int Nr, double dr, double fov, int pad, int Lmax, const int32_t* __restrict__ perm,
    const int32_t* __restrict__ psN, const int32_t* __restrict__ nrhoSorted,
    const int32_t* __restrict__ lineOffSorted, const double* __restrict__ cosTab,
    const float* __restrict__ taper, const double* __restrict__ w, double* __restrict__ part) {
  extern __shared__ double ps_smem[];
  const int j = j0 + blockIdx.x;
  const int N = psN[j];
  const int c = N / 2;
  const int L = pad * N;
  const int stride = Lmax / L;
  // groups of threads sharing one offset i split the sum over j
  const int G = c >= kPsThreads ? 1 : kPsThreads / c;
  const int span = c >= kPsThreads ? kPsThreads : c;  // offsets per pass
  double* cosL = ps_smem;                   // [L]
  double2* proj = (double2*)(ps_smem + L);  // [c]
  double2* partial = proj + c;              // [G][span]
  const int tid = threadIdx.x;
  for (int m = tid; m < L; m += kPsThreads) cosL[m] = cosTab[(size_t)m * stride];

  const double dl = fov / (double)N;
  const double wv = w[perm[j]];
  const int lane = tid % span;
  const int g = tid / span;
  for (int base = 0; base < c; base += span) {
    const int i = base + lane;
    if (g < G) {
      double re = 0.0, im = 0.0;
      for (int jj = g; jj < c; jj += G) {
        const int d2 = i * i + jj * jj;
        if (d2 >= c * c) break;  // d2 grows with jj
        const double r2 = (double)d2 * dl * dl;
        const double phi = r2 / (1.0 + sqrt(1.0 - r2));
        double t = wv * phi;
        t -= rint(t);
        double sn, cs;
        sincospi(2.0 * t, &sn, &cs);
        const double tau = taper_at(sqrt(r2), dr, Nr, taper);
        const double wt = jj == 0 ? 1.0 : 2.0;
        re += wt * tau * cs;
        im += wt * tau * sn;
      }
      partial[g * span + lane] = make_double2(re, im);
    }
    __syncthreads();
    if (tid < span) {
      double re = 0.0, im = 0.0;
      for (int gg = 0; gg < G; ++gg) {
        re += partial[gg * span + tid].x;
        im += partial[gg * span + tid].y;
      }
      proj[base + tid] = make_double2(re * dl, im * dl);
    }
    __syncthreads();
  }

  const int n = nrhoSorted[j];
  double* dst = part + (size_t)lineOffSorted[j] * 2;
  for (int k = tid; k < n; k += kPsThreads) {
    double re = 0.0, im = 0.0;
    int m = 0;  // k i mod L
    for (int i = 1; i < c; ++i) {
      m += k;
      if (m >= L) m -= L;
      const double cv = cosL[m];
      re += proj[i].x * cv;
      im += proj[i].y * cv;
    }
    dst[2 * k] = dl * (proj[0].x + 2.0 * re);
    dst[2 * k + 1] = dl * (proj[0].y + 2.0 * im);
  }
}


}  // namespace

// ------------------------------ launchers ---------------------------------
hipError_t launch_hankel_matrix(const DevPlan& p, hipStream_t s) {
  dim3 grid((p.NrPad + 255) / 256, p.rowsPad);
  hipLaunchKernelGGL(k_hankel_matrix, grid, dim3(256), 0, s, p.rowsPad, p.NrPad, p.Nr,
                     p.nrhoMax, p.dr, p.drho, p.M32, p.Msplit, p.MsplitG);
  return hipGetLastError();
}

constexpr int kScreenPlanes = 8;

hipError_t launch_screen(const DevPlan& p, int j0, int j1, const float* taper, const double* w,
                         ScreenLayout layout, hipStream_t s) {
  if (j1 <= j0) return hipSuccess;
  if (layout == kScreenGroups) {
    const int run = 64 * kScreenPlaneRun;
    dim3 grid((j1 - j0 + run - 1) / run, p.NrPad / 16);
    hipLaunchKernelGGL(k_screen_f32_groups, grid, dim3(256), 0, s, j0, j1, p.Nr, p.colsPad,
                       p.perm, p.phi, taper, w, p.B32);
  } else if (layout == kScreenColumns) {
    // about kScreenPlanes planes per workgroup
    const int want = (j1 - j0 + kScreenPlanes - 1) / kScreenPlanes;
    const int gy = want < 65535 ? want : 65535;
    dim3 grid((p.NrPad / 4 + 255) / 256, gy);
    hipLaunchKernelGGL(k_screen_f32, grid, dim3(256), 0, s, j0, j1, p.Nr, p.NrPad, p.perm, p.phi,
                       taper, w, p.B32);
  } else {
    const int gy = (j1 - j0) < 65535 ? (j1 - j0) : 65535;
    dim3 grid((p.NrPad / 8 + 255) / 256, gy);
    hipLaunchKernelGGL(k_screen_bf16, grid, dim3(256), 0, s, j0, j1, p.Nr, p.NrPad, p.perm,
                       p.phi, taper, w, p.Bsplit);
  }
  return hipGetLastError();
}

ContractShape contract_shape(int variant) {
  switch (variant) {
    case kWave32x64: return ContractShape{1, 64, 1};
    case kWave32x128: return ContractShape{1, 128, 1};
    case kLds128x128: return ContractShape{4, 128, 1};
    case kLds64x256: return ContractShape{2, 256, 1};
    case kRing128x128: return ContractShape{4, 128, 1};
    case kRing64x256: return ContractShape{2, 256, 1};
    case kRingF128x128: return ContractShape{4, 128, 1};
    case kRingF64x256: return ContractShape{2, 256, 1};
    case kRingF64x256W8: return ContractShape{2, 256, 1};
    case kRingH64x256: return ContractShape{2, 256, 1};
    case kRingR64x256: return ContractShape{2, 256, 1};
    case kRingW64x256: return ContractShape{2, 256, 1};
    default: return ContractShape{1, 512, 1};  // kRing32x512
  }
}

hipError_t launch_contract(const DevPlan& p, int variant, const Tile* tiles, int nTiles,
                           hipStream_t s) {
  if (nTiles <= 0) return hipSuccess;
  const dim3 g(nTiles);
  if (p.precision == 0) {
    const float4* A = (const float4*)p.M32;
    const float4* B = (const float4*)p.B32;
    switch (variant) {
      case kRingF128x128:
        hipLaunchKernelGGL((k_contract_f32_ringf<2, 2, 2, 2, 8>), g, dim3(256), 0, s, tiles,
                           p.NrPad, p.kchunk, p.P, p.lineTotal, p.M32, p.B32, p.nrhoSorted,
                           p.lineOffSorted, p.part);
        break;
      case kRingF64x256:
        hipLaunchKernelGGL((k_contract_f32_ringf<1, 4, 2, 2, 8>), g, dim3(256), 0, s, tiles,
                           p.NrPad, p.kchunk, p.P, p.lineTotal, p.M32, p.B32, p.nrhoSorted,
                           p.lineOffSorted, p.part);
        break;
      case kRingF64x256W8:
        hipLaunchKernelGGL((k_contract_f32_ringf<2, 4, 1, 2, 8>), g, dim3(512), 0, s, tiles,
                           p.NrPad, p.kchunk, p.P, p.lineTotal, p.M32, p.B32, p.nrhoSorted,
                           p.lineOffSorted, p.part);
        break;
      case kWave32x64:
        hipLaunchKernelGGL(k_contract_f32<2>, g, dim3(64), 0, s, tiles, p.NrPad, p.kchunk, p.P,
                           p.lineTotal, p.M32, p.B32, p.nrhoSorted, p.lineOffSorted, p.part);
        break;
      case kWave32x128:
        hipLaunchKernelGGL(k_contract_f32<4>, g, dim3(64), 0, s, tiles, p.NrPad, p.kchunk, p.P,
                           p.lineTotal, p.M32, p.B32, p.nrhoSorted, p.lineOffSorted, p.part);
        break;
      case kLds128x128:
        hipLaunchKernelGGL((k_contract_f32_lds<4, 1>), g, dim3(256), 0, s, tiles, p.NrPad,
                           p.kchunk, p.P, p.lineTotal, A, B, p.nrhoSorted, p.lineOffSorted,
                           p.part);
        break;
      case kLds64x256:
        hipLaunchKernelGGL((k_contract_f32_lds<2, 2>), g, dim3(256), 0, s, tiles, p.NrPad,
                           p.kchunk, p.P, p.lineTotal, A, B, p.nrhoSorted, p.lineOffSorted,
                           p.part);
        break;
      default:
        return hipErrorInvalidValue;  // no FP32 kernel for this variant
    }
  } else {
    const uint4* A = (const uint4*)p.Msplit;
    const uint4* B = (const uint4*)p.Bsplit;
    switch (variant) {
      case kWave32x64:
        hipLaunchKernelGGL(k_contract_bf16x6<2>, g, dim3(64), 0, s, tiles, p.NrPad, p.kchunk,
                           p.P, p.lineTotal, p.Msplit, p.Bsplit, p.nrhoSorted, p.lineOffSorted,
                           p.part);
        break;
      case kWave32x128:
        hipLaunchKernelGGL(k_contract_bf16x6<4>, g, dim3(64), 0, s, tiles, p.NrPad, p.kchunk,
                           p.P, p.lineTotal, p.Msplit, p.Bsplit, p.nrhoSorted, p.lineOffSorted,
                           p.part);
        break;
      case kLds128x128:
        hipLaunchKernelGGL((k_contract_bf16x6_lds<4, 1>), g, dim3(256), 0, s, tiles, p.NrPad,
                           p.kchunk, p.P, p.lineTotal, A, B, p.nrhoSorted, p.lineOffSorted,
                           p.part);
        break;
      case kLds64x256:
        hipLaunchKernelGGL((k_contract_bf16x6_lds<2, 2>), g, dim3(256), 0, s, tiles, p.NrPad,
                           p.kchunk, p.P, p.lineTotal, A, B, p.nrhoSorted, p.lineOffSorted,
                           p.part);
        break;
      case kRing128x128:
        hipLaunchKernelGGL((k_contract_bf16x6_ring<2, 2, 2, 2, 4>), g, dim3(256), 0, s, tiles,
                           p.NrPad, p.kchunk, p.P, p.lineTotal, A, B, p.nrhoSorted,
                           p.lineOffSorted, p.part);
        break;
      case kRing64x256:
        hipLaunchKernelGGL((k_contract_bf16x6_ring<1, 4, 2, 2, 4>), g, dim3(256), 0, s, tiles,
                           p.NrPad, p.kchunk, p.P, p.lineTotal, A, B, p.nrhoSorted,
                           p.lineOffSorted, p.part);
        break;
      case kRingF128x128:
        hipLaunchKernelGGL((k_contract_bf16x6_ringf<2, 2, 2, 2, 8>), g, dim3(256), 0, s, tiles,
                           p.NrPad, p.kchunk, p.P, p.lineTotal, p.M32, p.B32, p.nrhoSorted,
                           p.lineOffSorted, p.part);
        break;
      case kRingF64x256:
        hipLaunchKernelGGL((k_contract_bf16x6_ringf<1, 4, 2, 2, 8>), g, dim3(256), 0, s, tiles,
                           p.NrPad, p.kchunk, p.P, p.lineTotal, p.M32, p.B32, p.nrhoSorted,
                           p.lineOffSorted, p.part);
        break;
      case kRingF64x256W8:
        hipLaunchKernelGGL((k_contract_bf16x6_ringf<2, 4, 1, 2, 8>), g, dim3(512), 0, s, tiles,
                           p.NrPad, p.kchunk, p.P, p.lineTotal, p.M32, p.B32, p.nrhoSorted,
                           p.lineOffSorted, p.part);
        break;
      case kRingH64x256:
        if (!p.MsplitG) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_contract_bf16x6_ringh<7>), g, dim3(512), 0, s, tiles, p.NrPad,
                           p.rowsPad, p.kchunk, p.P, p.lineTotal, (const uint4*)p.MsplitG, p.B32,
                           p.nrhoSorted, p.lineOffSorted, p.part);
        break;
      case kRingR64x256:
        if (!p.MsplitG) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_contract_bf16x6_ringr, g, dim3(512), 0, s, tiles, p.NrPad,
                           p.rowsPad, p.kchunk, p.P, p.lineTotal, (const uint4*)p.MsplitG, p.B32,
                           p.nrhoSorted, p.lineOffSorted, p.part);
        break;
      case kRingW64x256:
        if (!p.MsplitG) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_contract_bf16x6_ringw, g, dim3(512), 0, s, tiles, p.colsPad,
                           p.rowsPad, p.kchunk, p.P, p.lineTotal, (const uint4*)p.MsplitG, p.B32,
                           p.nrhoSorted, p.lineOffSorted, p.part);
        break;
      default:
        hipLaunchKernelGGL((k_contract_bf16x6_ring<1, 4, 1, 4, 3>), g, dim3(256), 0, s, tiles,
                           p.NrPad, p.kchunk, p.P, p.lineTotal, A, B, p.nrhoSorted,
                           p.lineOffSorted, p.part);
        break;
    }
  }
  return hipGetLastError();
}

hipError_t launch_spline(const DevPlan& p, int j0, int j1, hipStream_t s, double frac,
                         int32_t* hTrunc) {
  // Planes are sorted by radial length (longest first); each launch covers a
  // run of planes whose lines fit its LDS size, so short lines are not
  // limited to the occupancy of the longest one.
  static const int kBucket[] = {kMaxRho, 512, 128, 48};
  for (int b = 0; b < 4 && j0 < j1; ++b) {
    const int cap = kBucket[b];
    const int nextCap = b + 1 < 4 ? kBucket[b + 1] : 0;
    int jb = j0;
    while (jb < j1 && p.nrhoSortedHost[jb] > nextCap) ++jb;
    if (jb == j0) continue;
    const int nmax = p.nrhoSortedHost[j0] < cap ? p.nrhoSortedHost[j0] : cap;
    const size_t shm = (size_t)3 * nmax * sizeof(double2);
    hipLaunchKernelGGL(k_spline, dim3(jb - j0), dim3(64), shm, s, j0, p.nkc, p.lineTotal,
                       p.interp, p.nrhoSorted, p.lineOffSorted, p.cprime, p.part, p.coef,
                       frac * frac, p.q * p.os, hTrunc, p.perm, p.status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    j0 = jb;
  }
  return hipSuccess;
}

hipError_t prepare_kernels(const DevPlan& p) {
  // dynamic LDS above 64 KiB must be enabled per kernel before any launch
  // (and before any stream capture)
  const size_t shmSpline = (size_t)3 * p.nrhoMax * sizeof(double2);
  if (shmSpline > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_spline,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmSpline);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_ps_lines(const DevPlan& p, const PsTables& t, int j0, int j1,
                           const float* taper, const double* w, hipStream_t s) {
  if (j1 <= j0) return hipSuccess;
  const int c = t.maxN / 2;
  const int span = c >= kPsThreads ? kPsThreads : c;
  const int G = c >= kPsThreads ? 1 : kPsThreads / c;
  const size_t shm = (size_t)t.Lmax * sizeof(double) + (size_t)c * sizeof(double2) +
                     (size_t)G * span * sizeof(double2);
  if (shm > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_ps_lines,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_ps_lines, dim3(j1 - j0), dim3(kPsThreads), shm, s, j0, p.Nr, p.dr, t.fov,
                     p.q * p.os, t.Lmax, p.perm, t.n, p.nrhoSorted, p.lineOffSorted, t.cosTab,
                     taper, w, p.part);
  return hipGetLastError();
}


hipError_t launch_lines_out(const DevPlan& p, void* lines, hipStream_t s) {
  dim3 grid(4, p.Pall);
  hipLaunchKernelGGL(k_lines_out, grid, dim3(256), 0, s, p.Pall, p.nkc, p.lineTotal, p.planes,
                     p.part, (double2*)lines);
  return hipGetLastError();
}

hipError_t launch_grad(const DevPlan& p, const GradScratch& gs, const float* taper,
                       const double* w, const void* gout, float* gtau, double* gw,
                       hipStream_t s) {
  // samples of one interval: at most the lattice points of its ring (radius
  // (k + 1) / q at most, width 1 / q, widened for the radius rounding)
  const double rq = (double)p.nrhoMax / p.q;
  const double ringPts = M_PI * (2.0 * rq / p.q + 2e-6 * rq * rq + 2.0) + 4.0 * M_PI * (rq + 1.0) +
                         M_PI + 16.0;
  const int eN = (int)std::ceil(std::log2(ringPts));
  const int64_t n8 = (int64_t)p.lineTotalAll * 8;
  hipLaunchKernelGGL(k_grad_clear, dim3(1024), dim3(256), 0, s, n8, gs.momfx, p.Pall, gs.amax);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_grad_absmax, dim3(p.nUnits), dim3(256), 0, s, p.units, p.planes,
                     (const float2*)gout, gs.amax);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t shm = (size_t)p.nrhoMax * 8 * sizeof(unsigned long long);
  if (shm > 65536) {
    e = hipFuncSetAttribute((const void*)k_resample_T, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)shm);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_resample_T, dim3(p.nUnits), dim3(kMomThreads), shm, s, p.units, p.planes,
                     p.os, 1.0f / (float)p.os, (float)p.q, eN, gs.amax, (const float2*)gout,
                     gs.momfx);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_mom_convert, dim3((p.nrhoMax + 255) / 256, p.Pall), dim3(256), 0, s,
                     p.planes, eN, gs.amax, gs.momfx, gs.mom);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t shmT = (size_t)3 * p.nrhoMax * sizeof(double2);
  if (shmT > 65536) {
    e = hipFuncSetAttribute((const void*)k_spline_T, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)shmT);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_spline_T, dim3(p.P), dim3(64), shmT, s, 0, p.interp, p.perm,
                     p.nrhoSorted, p.lineOffSorted, p.lineOffCaller, p.mirStart, p.mirList,
                     p.cprime, gs.mom, gs.gy);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  dim3 g3((p.Nr + 255) / 256, p.P);
  hipLaunchKernelGGL(k_contract_T, g3, dim3(256), 0, s, p.Nr, p.NrPad, p.perm, p.nrhoSorted,
                     p.lineOffSorted, p.M32, p.phi, taper, w, gs.gy, gs.ure, gs.wterm);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_grad_taper, dim3((p.Nr + 31) / 32), dim3(256), 0, s, p.P, p.Nr, p.NrPad,
                     gs.ure, gtau);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_grad_w, dim3(p.P), dim3(256), 0, s, p.Nr, p.NrPad, p.perm, gs.wterm, gw);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int nm = p.Pall - p.P;
  if (nm > 0) {
    hipLaunchKernelGGL(k_grad_w_mirrored, dim3((nm + 255) / 256), dim3(256), 0, s, nm, p.mirList,
                       gw);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace wkern
