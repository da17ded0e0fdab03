// Resample of the radial lines into the oversampled kernel cache (section
// 4.4, Algorithm 2) and the truncated layout (section 3.1).
#include "wkern_internal.h"
#include "wkern_radial.h"

namespace wkern {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// --------------------------------------------------------------------------
// Oversampled kernel cache (section 4.4, Algorithm 2), element
// e = ((fv os + fu) S + b) S + a of a plane.  Full cache: a workgroup of 256
// threads per resample unit (at most kUnitElems consecutive elements of one
// plane, starting at a multiple of 1024), the plane's spline intervals staged
// in LDS once; the truncated layout writes its units the same way.  Each wave takes 128
// consecutive elements per step (waves interleaved, 512 per step) and each
// lane two neighbours, written with one 16-byte store: on this chip that
// store pattern writes the cache about 8% faster than one 8-byte store per
// element.  A wave decodes its first element once with scalar divisions and
// advances it by 512 elements a step with scalar carries; for S >= 64 the
// 128 elements span at most three rows, so a lane's X is its column-0 X plus
// os times its offset, less a wave-uniform amount past each row boundary,
// and Y^2 is one of three wave-uniform values.  The radial position is the
// same FP32 computation as radial_pos (sq rounded before it is used, the
// halving of the Newton correction folded into q / 2, d2 = 0 through the
// max), so the cache is bit-identical to what cache_value gives.
// --------------------------------------------------------------------------
template <bool kQ1>
__device__ __forceinline__ f32x2 unit_value(int d2, int lim, float q, float hq, int nmax,
                                            const float4* __restrict__ sc, uint32_t sgn) {
  const float d2f = (float)d2;
  const float rs = __builtin_amdgcn_rsqf(fmaxf(d2f, 1.0f));
  const float sq = __fmul_rn(d2f, rs);
  const float c = __fmul_rn(fmaf(-sq, sq, d2f), rs);
  // q = 1: q sq is sq exactly.  fma(q, sq, -k) keeps q as a run-time
  // operand: with q folded to 1 the compiler would form sq - k as
  // fma(rs, d2f, -k), skipping the rounding of sq that radial_pos has.
  const int k = min((int)(kQ1 ? sq : q * sq), nmax);
  const float uu = fmaf(hq, c, fmaf(q, sq, -(float)k));
  const int kk = d2 <= lim ? k : nmax + 1;  // interval nmax + 1 is zero
  const float4 cr = sc[2 * kk];
  const float4 ci = sc[2 * kk + 1];
  f32x2 v;
  v.x = fmaf(uu, fmaf(uu, fmaf(uu, cr.w, cr.z), cr.y), cr.x);
  v.y = __uint_as_float(__float_as_uint(fmaf(uu, fmaf(uu, fmaf(uu, ci.w, ci.z), ci.y), ci.x)) ^
                        sgn);
  return v;
}

// Wave-uniform position of the first element of a step: column a of row b
// of sub-kernel (fu, fv), with the carries of one row.
struct RowPos {
  int a, b, fu, fv;
};
// The row after p's (column unchanged).
__device__ __forceinline__ RowPos next_row(RowPos p, int S, int os) {
  const int wb = (int)(p.b + 1 == S);
  const int fu = p.fu + wb;
  const int wf = (int)(fu == os);
  return RowPos{p.a, (p.b + 1) * (1 - wb), fu - wf * os, p.fv + wf};
}
// p advanced by stepR rows and stepA columns (stepR < S, stepA < S).
__device__ __forceinline__ RowPos advance(RowPos p, int stepR, int stepA, int S, int os) {
  const int ca = (int)(p.a + stepA >= S);
  const int bb = p.b + stepR + ca;
  const int wb = (int)(bb >= S);
  const int fu = p.fu + wb;
  const int wf = (int)(fu == os);
  return RowPos{p.a + stepA - ca * S, bb - wb * S, fu - wf * os, p.fv + wf};
}

// Elements [e, e1) of a plane with S >= 64.  Each wave takes kChunk
// consecutive elements per step (the block's 4 waves interleaved, 4 kChunk
// per step), each lane kChunk / 64 of them as pairs written with 16-byte
// stores.  The chunk spans at most three rows (kChunk = 256 needs S >= 128,
// kChunk = 128 needs S >= 64); the rows' column-0 X and Y^2 are
// wave-uniform (scalar registers) and a lane's X is column-0 X plus os times
// its offset, less a uniform amount past each row boundary.  A chunk that
// lies wholly before e1 is stored without per-element checks.
template <int kChunk, bool kQ1>
__device__ __forceinline__ void resample_rows(int e, int e1, RowPos p0, int S, int h, int os,
                                              int lim, float q, float hq, int nmax,
                                              const float4* __restrict__ sc, uint32_t sgn,
                                              int off, bool al16, f32x2* __restrict__ o) {
  constexpr int kPairs = kChunk / 128;  // 16-byte stores per lane per step
  const int step = 4 * kChunk;
  const int stepR = step / S, stepA = step - stepR * S;
  const int xoff = __mul24(os, off);
  for (; e < e1; e += step) {
    const RowPos p1 = next_row(p0, S, os), p2 = next_row(p1, S, os);
    const int x0 = os * (p0.a - h) - p0.fu;
    const int Y0 = os * (p0.b - h) - p0.fv, Y1 = os * (p1.b - h) - p1.fv,
              Y2 = os * (p2.b - h) - p2.fv;
    const int y0 = Y0 * Y0, dy1 = Y1 * Y1 - y0, dy2 = Y2 * Y2 - y0;
    const int dx1 = os * S + p1.fu - p0.fu, dx2 = 2 * os * S + p2.fu - p0.fu;
    const int S1 = S - p0.a, S2 = 2 * S - p0.a;  // first offsets in rows 1 and 2
    auto d2_at = [=](int t, int xt) {
      const bool r1 = t >= S1, r2 = t >= S2;
      const int X = xt - (r2 ? dx2 : (r1 ? dx1 : 0));
      return __mul24(X, X) + y0 + (r2 ? dy2 : (r1 ? dy1 : 0));
    };
    const bool full = e + kChunk <= e1 && al16;  // wave-uniform
#pragma unroll
    for (int k = 0; k < kPairs; ++k) {
      const int t = off + 128 * k;
      const int xt = x0 + xoff + 128 * k * os;
      const f32x2 v0 = unit_value<kQ1>(d2_at(t, xt), lim, q, hq, nmax, sc, sgn);
      const f32x2 v1 = unit_value<kQ1>(d2_at(t + 1, xt + os), lim, q, hq, nmax, sc, sgn);
      const int ee = e + t;
      f32x2* p = o + ee;
      if (full) {
        f32x4 w4 = {v0.x, v0.y, v1.x, v1.y};
        *(f32x4*)p = w4;
      } else {
        if (ee < e1) p[0] = v0;
        if (ee + 1 < e1) p[1] = v1;
      }
    }
    p0 = advance(p0, stepR, stepA, S, os);
  }
}

// Elements [e0, e1) of plane pi (its spline intervals in sc), by the block's
// 4 waves; e0 is even.
template <bool kQ1>
__device__ __forceinline__ void resample_unit(const PlaneInfo& pi, int e0, int e1, int os,
                                              float invOs, uint32_t magicOs, int shiftOs,
                                              float q, const float4* __restrict__ sc,
                                              float2* __restrict__ out) {
  const int S = pi.S, h = pi.h, lim = pi.lim;
  const int nmax = pi.nrho - 2;
  const float hq = 0.5f * q;
  const uint32_t sgn = pi.conj ? 0x80000000u : 0u;
  const int off = 2 * (threadIdx.x & 63);
  f32x2* const o = (f32x2*)(out + pi.out_off);
  const bool al16 = ((uintptr_t)o & 15) == 0;
  if (S >= 64) {
    // scalar decode of the first element of the wave's first chunk
    const int ch = S >= 128 ? 256 : 128;
    const int w0 = e0 + ch * __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int R = (int)(__umulhi((uint32_t)w0, pi.magicS) >> pi.shiftS);
    const int F = (int)(__umulhi((uint32_t)R, pi.magicS) >> pi.shiftS);
    const int fv = os == 1 ? F : (int)(__umulhi((uint32_t)F, magicOs) >> shiftOs);
    const RowPos p0{w0 - R * S, R - F * S, F - fv * os, fv};
    if (S >= 128)
      resample_rows<256, kQ1>(w0, e1, p0, S, h, os, lim, q, hq, nmax, sc, sgn, off, al16, o);
    else
      resample_rows<128, kQ1>(w0, e1, p0, S, h, os, lim, q, hq, nmax, sc, sgn, off, al16, o);
  } else {
    const int e = e0 + 128 * __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int ee = e + off; ee - off < e1; ee += 512) {
      // the pair's first element by division, the second by one column step
      // with the carries into row, fu and fv
      int a, b, fu;
      const int R = div_small(ee, S, pi.invS, a);
      const int F = div_small(R, S, pi.invS, b);
      int fv = div_small(F, os, invOs, fu);
      const int X0 = os * (a - h) - fu;
      const int Y0 = os * (b - h) - fv;
      if (++a == S) {
        a = 0;
        if (++b == S) {
          b = 0;
          if (++fu == os) {
            fu = 0;
            ++fv;
          }
        }
      }
      const int X1 = os * (a - h) - fu;
      const int Y1 = os * (b - h) - fv;
      const f32x2 v0 =
          unit_value<kQ1>(__mul24(X0, X0) + __mul24(Y0, Y0), lim, q, hq, nmax, sc, sgn);
      const f32x2 v1 =
          unit_value<kQ1>(__mul24(X1, X1) + __mul24(Y1, Y1), lim, q, hq, nmax, sc, sgn);
      f32x2* p = o + ee;
      if (ee + 1 < e1 && al16) {
        f32x4 w4 = {v0.x, v0.y, v1.x, v1.y};
        *(f32x4*)p = w4;
      } else {
        if (ee < e1) p[0] = v0;
        if (ee + 1 < e1) p[1] = v1;
      }
    }
  }
}

template <bool kQ1>
__global__ __launch_bounds__(256) void k_resample(const ResampleUnit* __restrict__ units,
                                                  int nUnits,
                                                  const PlaneInfo* __restrict__ planes,
                                                  const float4* __restrict__ coef, int os,
                                                  float invOs, uint32_t magicOs, int shiftOs,
                                                  float q, float2* __restrict__ out) {
  // Interval j's re and im coefficients at sc[2 j], sc[2 j + 1].  Interval
  // nrho - 1 (never a sample's) is zeroed and serves the samples outside the
  // support.
  extern __shared__ float4 sc[];  // [nrho][2]
  // Workgroups go to the XCDs in turn, so workgroup b runs on XCD b mod 8
  // as its slot-th workgroup there (slot = b / 8).  The units are cut into
  // runs of kXcdRun consecutive units, dealt to the XCDs in turn: XCD x
  // takes runs x, x + 8, ..., and walks each in address order.  A plane's
  // units then mostly share one XCD, and its intervals are fetched into
  // that XCD's L2 once instead of once per XCD (the same cache bytes).  With
  // the intervals local, shorter units pay: see kUnitElems.  Runs of 64
  // units (16 MB) measured best: on two boxes 5.396-5.403 and 5.540-5.552
  // ms against 5.424-5.428 and 5.591-5.604 with one contiguous eighth per
  // XCD; runs of 16, 32, 128 or 512 units were slower than either.  (The
  // truncated layout's small units measured faster in plain address order,
  // 1.13 against 1.18 ms per truncated call.)
  const int slot = (int)(blockIdx.x / kNumXcd), xcd = (int)(blockIdx.x % kNumXcd);
  const int ui = ((slot / kXcdRun) * kNumXcd + xcd) * kXcdRun + slot % kXcdRun;
  if (ui >= nUnits) return;
  const ResampleUnit u = units[ui];
  const PlaneInfo pi = planes[u.p];
  const int nmax = pi.nrho - 2;
  const float4* src = coef + (size_t)pi.line_off * 2;
  for (int i = threadIdx.x; i < 2 * nmax + 2; i += 256) sc[i] = src[i];
  if (threadIdx.x < 2) sc[2 * nmax + 2 + threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
  __syncthreads();
  resample_unit<kQ1>(pi, u.e0, u.e1, os, invOs, magicOs, shiftOs, q, sc, out);
}

// Truncated layout (section 3.1, Algorithm 2): one block of 1024 threads.
// Plane p (caller order) takes the half-width its source line was truncated
// to; writes supports, the exclusive prefix sums of os^2 S^2 (offsets) and
// of the per-plane resample units (unitStart, units of kUnitElems), and the
// plane of every unit (unitPlane).  Thread t sums a run of consecutive
// planes, one scan over the 1024 run totals gives each run its start, and
// the thread then writes its planes' entries (integer sums: the same result
// in any order).
__global__ __launch_bounds__(1024) void k_trunc_layout(int Pall, int os,
                                                       const int32_t* __restrict__ hSorted,
                                                       const int32_t* __restrict__ sortedPos,
                                                       int32_t* __restrict__ supportOut,
                                                       int64_t* __restrict__ offsetsOut,
                                                       int32_t* __restrict__ unitStart,
                                                       int32_t* __restrict__ unitPlane) {
  __shared__ int64_t sBytes[1024];
  __shared__ int32_t sUnits[1024];
  extern __shared__ uint16_t sWidth[];  // [Pall] truncated widths (<= 4095)
  const int t = (int)threadIdx.x;
#pragma unroll 8
  for (int p = t; p < Pall; p += 1024) sWidth[p] = (uint16_t)(2 * hSorted[sortedPos[p]] + 1);
  __syncthreads();
  const int per = (Pall + 1023) / 1024;
  const int p0 = min(Pall, t * per), p1 = min(Pall, p0 + per);
  auto width = [&](int p) { return (int)sWidth[p]; };
  int64_t nb = 0;
  int32_t nu = 0;
  for (int p = p0; p < p1; ++p) {
    const int S = width(p);
    const int64_t n = (int64_t)os * os * S * S;
    nb += n;
    nu += (int32_t)((n + kUnitElems - 1) / kUnitElems);
  }
  sBytes[t] = nb;
  sUnits[t] = nu;
  __syncthreads();
  // inclusive scan (Hillis-Steele) over the run totals
  for (int d = 1; d < 1024; d <<= 1) {
    int64_t tb = 0;
    int32_t tu = 0;
    if (t >= d) {
      tb = sBytes[t - d];
      tu = sUnits[t - d];
    }
    __syncthreads();
    sBytes[t] += tb;
    sUnits[t] += tu;
    __syncthreads();
  }
  int64_t cb = sBytes[t] - nb;
  int32_t cu = sUnits[t] - nu;
  for (int p = p0; p < p1; ++p) {
    const int S = width(p);
    const int64_t n = (int64_t)os * os * S * S;
    const int32_t k = (int32_t)((n + kUnitElems - 1) / kUnitElems);
    supportOut[p] = S;
    offsetsOut[p] = cb;
    unitStart[p] = cu;
    for (int32_t i = 0; i < k; ++i) unitPlane[cu + i] = p;
    cb += n;
    cu += k;
  }
  if (t == 1023) {
    offsetsOut[Pall] = sBytes[1023];
    unitStart[Pall] = sUnits[1023];
  }
}

// Resample of a truncated layout: a fixed grid walks the units; unit u
// belongs to plane unitPlane[u].  The plane's entry takes its truncated
// width (and the divisors for it), and the unit is written as in the full
// cache.
template <bool kQ1>
__global__ __launch_bounds__(256) void k_resample_trunc(int Pall, const PlaneInfo* __restrict__ planes,
                                                        const int32_t* __restrict__ supportOut,
                                                        const int64_t* __restrict__ offsetsOut,
                                                        const int32_t* __restrict__ unitStart,
                                                        const int32_t* __restrict__ unitPlane,
                                                        const float4* __restrict__ coef, int os,
                                                        float invOs, uint32_t magicOs, int shiftOs,
                                                        float q, float2* __restrict__ out) {
  extern __shared__ float4 sc[];
  const int total = unitStart[Pall];
  const int qi = (int)q;
  for (int u = blockIdx.x; u < total; u += gridDim.x) {
    const int p = unitPlane[u];
    PlaneInfo pi = planes[p];
    const int S = supportOut[p];
    pi.S = S;
    pi.h = (S - 1) / 2;
    pi.lim = (os * pi.h) * (os * pi.h);
    pi.invS = 1.0f / (float)S;
    pi.out_off = offsetsOut[p];
    magic_div24((uint32_t)(S > 2 ? S : 2), pi.magicS, pi.shiftS);
    const int n = os * os * S * S;
    const int e0 = (u - unitStart[p]) * kUnitElems;
    const int e1 = min(n, e0 + kUnitElems);
    const int nmax = pi.nrho - 2;
    // a sample inside the truncated support has q sqrt(d2) <= q os h, so it
    // reads an interval up to q os h; the line runs to the planned support,
    // and only its first intervals are staged (plus the zero interval
    // nmax + 1 for the samples outside)
    const int kTop = min(nmax, qi * os * pi.h + 1);
    __syncthreads();  // the previous unit is done with sc
    const float4* src = coef + (size_t)pi.line_off * 2;
    for (int k = threadIdx.x; k < 2 * kTop + 2; k += 256) sc[k] = src[k];
    if (threadIdx.x < 2) sc[2 * nmax + 2 + threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    resample_unit<kQ1>(pi, e0, e1, os, invOs, magicOs, shiftOs, q, sc, out);
  }
}

}  // namespace

hipError_t launch_resample(const DevPlan& p, int u0, int u1, void* out, hipStream_t s) {
  if (u1 <= u0) return hipSuccess;
  const size_t shm = (size_t)2 * p.nrhoMax * sizeof(float4);
  uint32_t mOs = 0;
  int32_t shOs = 0;
  if (p.os >= 2) magic_div24((uint32_t)p.os, mOs, shOs);
  const int n = u1 - u0;
  // workgroups per XCD: whole runs of kXcdRun units
  const int per = (n + kNumXcd * kXcdRun - 1) / (kNumXcd * kXcdRun) * kXcdRun;
  if (p.q == 1)
    hipLaunchKernelGGL(k_resample<true>, dim3(per * kNumXcd), dim3(256), shm, s, p.units + u0,
                       n, p.planes, p.coef, p.os, 1.0f / (float)p.os, mOs, shOs, 1.0f,
                       (float2*)out);
  else
    hipLaunchKernelGGL(k_resample<false>, dim3(per * kNumXcd), dim3(256), shm, s, p.units + u0,
                       n, p.planes, p.coef, p.os, 1.0f / (float)p.os, mOs, shOs,
                       (float)p.q, (float2*)out);
  return hipGetLastError();
}

hipError_t prepare_resample_kernels(const DevPlan& p) {
  // the layout kernel holds every plane's width in LDS (2 bytes each) beside
  // 12 KB of scan arrays; above 64 KiB in all it must be enabled before any
  // launch or stream capture
  const size_t shmW = (size_t)p.Pall * sizeof(uint16_t);
  if (shmW > 65536 - 12288)
    return hipFuncSetAttribute((const void*)k_trunc_layout,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmW);
  return hipSuccess;
}

hipError_t launch_resample_truncated(const DevPlan& p, const TruncScratch& ts, double frac,
                                     int32_t* supportOut, int64_t* offsetsOut, void* out,
                                     hipStream_t s) {
  hipError_t e = launch_spline(p, 0, p.P, s, frac, ts.hTrunc);
  if (e != hipSuccess) return e;
  const size_t shmW = (size_t)p.Pall * sizeof(uint16_t);
  hipLaunchKernelGGL(k_trunc_layout, dim3(1), dim3(1024), shmW, s, p.Pall, p.os, ts.hTrunc,
                     ts.sortedPos, supportOut, offsetsOut, ts.unitStart, ts.unitPlane);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t shm = (size_t)2 * p.nrhoMax * sizeof(float4);
  uint32_t mOs = 0;
  int32_t shOs = 0;
  if (p.os >= 2) magic_div24((uint32_t)p.os, mOs, shOs);
  if (p.q == 1)
    hipLaunchKernelGGL(k_resample_trunc<true>, dim3(p.nUnits), dim3(256), shm, s, p.Pall, p.planes,
                       supportOut, offsetsOut, ts.unitStart, ts.unitPlane, p.coef, p.os, 1.0f / (float)p.os,
                       mOs, shOs, 1.0f, (float2*)out);
  else
    hipLaunchKernelGGL(k_resample_trunc<false>, dim3(p.nUnits), dim3(256), shm, s, p.Pall, p.planes,
                       supportOut, offsetsOut, ts.unitStart, ts.unitPlane, p.coef, p.os, 1.0f / (float)p.os,
                       mOs, shOs, (float)p.q, (float2*)out);
  return hipGetLastError();
}

}  // namespace wkern
