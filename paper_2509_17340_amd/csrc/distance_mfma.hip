// Pass A of the nearest-distance computation on the matrix cores (two variants).
//
// Built with finite-math (every value here is a finite squared distance or a
// finite padding constant), so that chained fminf become v_min3_f32 without
// NaN canonicalisation, and with MFMA results in VGPRs (no accumulator-register
// reads); the compiler inserts the MFMA-to-VALU wait states.  Both kernels write
// the same outputs as the VALU pass A: a per-query value, combined across cloud
// chunks with atomicMin on float bits, that is exact up to the stated rounding
// for every pair closer than d_max, and a per-block bound for the flag kernel.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "aero_device.h"
#include "aero_internal.h"

namespace aero {
namespace {

constexpr float kFarT = 1.0e30f;  // padding of the expanded form

// Pass A on the matrix cores.  t(point i, query j) = [-2 o'_i, |o'_i|^2] . [p'_j, 1] is a
// K = 4 contraction: one v_mfma_f32_16x16x4f32 per 16 points x 16 queries (lane l supplies
// A[l % 16][l / 16] = component l/16 of point l%16, B[l / 16][l % 16] = component l/16 of
// query l%16, and receives D rows 4 (l / 16) .. +3 of column l % 16).  Each wave holds
// kMfmaCols column blocks of 16 queries; the VALU only keeps the running minima.
constexpr int kMfmaCols = 8;
constexpr int kMfmaQPB = 4 * 64 / 4 * kMfmaCols;  // 4 waves x 16 queries x kMfmaCols = 512
typedef float floatx4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kBlock) void k_min_dist_approx_mfma(const QuerySet* __restrict__ sets,
                                                                 int n_sets) {
  __shared__ float4 tile[kTilePts];
  __shared__ float red[7][4];
  const int64_t bid = blockIdx.x;
  const int s = find_owner(sets, n_sets, bid, [](const QuerySet& q) { return q.block_base; });
  const QuerySet S = sets[s];
  const int64_t local = bid - S.block_base;
  const int qb = (int)(local / S.n_chunks), ch = (int)(local % S.n_chunks);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int col = lane & 15, kg = lane >> 4;
  float px[kMfmaCols], py[kMfmaCols], pz[kMfmaCols];
  bool ok[kMfmaCols];
  int32_t sid[kMfmaCols];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
#pragma unroll
  for (int b = 0; b < kMfmaCols; ++b) {
    const int64_t slot = (int64_t)qb * kMfmaQPB + w * (16 * kMfmaCols) + b * 16 + col;
    ok[b] = slot < S.Q;
    const int64_t qs = ok[b] ? slot : 0;  // positions in slot order
    sid[b] = (int32_t)slot;
    px[b] = S.sp[qs];
    py[b] = S.sp[S.Q + qs];
    pz[b] = S.sp[2 * S.Q + qs];
    if (ok[b]) {
      lo[0] = fminf(lo[0], px[b]);
      lo[1] = fminf(lo[1], py[b]);
      lo[2] = fminf(lo[2], pz[b]);
      hi[0] = fmaxf(hi[0], px[b]);
      hi[1] = fmaxf(hi[1], py[b]);
      hi[2] = fmaxf(hi[2], pz[b]);
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = wave_minf(lo[a]);
    hi[a] = wave_maxf(hi[a]);
  }
  if (lane == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      red[a][w] = lo[a];
      red[3 + a][w] = hi[a];
    }
  }
  __syncthreads();
  float c[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float l = fminf(fminf(red[a][0], red[a][1]), fminf(red[a][2], red[a][3]));
    const float h = fmaxf(fmaxf(red[3 + a][0], red[3 + a][1]), fmaxf(red[3 + a][2], red[3 + a][3]));
    c[a] = 0.5f * l + 0.5f * h;
  }
  float bop[kMfmaCols], pp[kMfmaCols], tmin[kMfmaCols], rr = 0.0f;
#pragma unroll
  for (int b = 0; b < kMfmaCols; ++b) {
    const float x = px[b] - c[0], y = py[b] - c[1], z = pz[b] - c[2];
    pp[b] = fmaf(z, z, fmaf(y, y, x * x));
    if (ok[b]) rr = fmaxf(rr, pp[b]);
    bop[b] = !ok[b] ? 0.0f : kg == 0 ? x : kg == 1 ? y : kg == 2 ? z : 1.0f;
    tmin[b] = kFarT;
  }
  // the MFMA sums four products per entry; the bound below (the same as the VALU
  // pass) covers that rounding with a wide margin
  rr = wave_maxf(rr);
  if (lane == 0) red[6][w] = rr;
  __syncthreads();
  const float R2 = fmaxf(fmaxf(red[6][0], red[6][1]), fmaxf(red[6][2], red[6][3]));
  const float span = sqrtf(R2) * 1.001f + S.d_max;
  const float thr = S.d_max * S.d_max + 0x1p-17f * span * span + 1e-6f;
  if (tid == 0 && ch == 0) {
    S.thresh[qb] = thr;
    S.seg_count[qb] = 0;
  }
  const floatx4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
  const float* tf = reinterpret_cast<const float*>(tile);
  const int64_t g0 = (int64_t)ch * S.chunk_pts;
  const int64_t g1 = min<int64_t>(g0 + S.chunk_pts, S.n_points);
  for (int64_t base = g0; base < g1; base += kTilePts) {
    const int cnt = (int)min<int64_t>(kTilePts, g1 - base);
    const int cnt16 = (cnt + 15) & ~15;  // groups of 16 points, padded
    for (int pt = tid; pt < cnt16; pt += kBlock) {
      const bool in = pt < cnt;
      const int64_t gg = in ? base + pt : base;
      const float ox = S.cloud[3 * gg] - c[0];
      const float oy = S.cloud[3 * gg + 1] - c[1];
      const float oz = S.cloud[3 * gg + 2] - c[2];
      tile[pt] = in ? make_float4(-2.0f * ox, -2.0f * oy, -2.0f * oz,
                                  fmaf(oz, oz, fmaf(oy, oy, ox * ox)))
                    : make_float4(0.0f, 0.0f, 0.0f, kFarT);
    }
    __syncthreads();
    float tt[kMfmaCols];
#pragma unroll
    for (int b = 0; b < kMfmaCols; ++b) tt[b] = kFarT;
#pragma unroll 2
    for (int g = 0; g < cnt16; g += 16) {
      const float a = tf[(g + col) * 4 + kg];
#pragma unroll
      for (int b = 0; b < kMfmaCols; ++b) {
        const floatx4 dv = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bop[b], zero, 0, 0, 0);
        tt[b] = fminf(tt[b], fminf(fminf(dv[0], dv[1]), fminf(dv[2], dv[3])));
      }
    }
    bool hit = false;
#pragma unroll
    for (int b = 0; b < kMfmaCols; ++b) {
      hit |= ok[b] && pp[b] + tt[b] < thr;
      tmin[b] = fminf(tmin[b], tt[b]);
    }
    if (__syncthreads_or(hit) && tid == 0)
      append_block_hits(S, qb, base / kTilePts, red, pass_b_reach2(thr, S.d_max));
  }
#pragma unroll
  for (int b = 0; b < kMfmaCols; ++b) {
    float v = tmin[b];
    v = fminf(v, __shfl_xor(v, 16, 64));
    v = fminf(v, __shfl_xor(v, 32, 64));
    if (ok[b] && kg == 0) atomicMin(S.out_slot + sid[b], __float_as_uint(fmaxf(pp[b] + v, 0.0f)));
  }
}

// Pass A on the half-precision matrix cores with near-single accuracy.  Every
// recentred coordinate is split into two halves, v = hi + lo (hi = half(v),
// lo = half(v - hi)), and one v_mfma_f32_32x32x16_f16 evaluates, for 32 cloud
// points x 32 queries,
//   t = n_hi + n_lo - 2 (o_hi.p_hi + o_lo.p_hi + o_hi.p_lo + o_lo.p_lo)
// with the K = 16 slots laid out as
//   A (point)  [-2o_hi, n_hi, -2o_lo, n_lo | -2o_hi, n_hi, -2o_lo, n_lo]
//   B (query)  [  p_hi,    1,   p_hi,    1 |   p_lo,    0,   p_lo,    0]
// (the zero query slots cancel the repeated norms, so both lane halves read the
// same 16-byte point record from LDS).  Half products are exact in the
// single-precision accumulator, so t carries the split error (2^-22 relative per
// coordinate) plus the accumulation rounding; the bound below is four times the
// single-precision passes' one.  Halves cover
// |v| < 65504: points with |o'| >= 128 become the constant t = 32768 (never
// flagged; they are provably farther than d_max whenever R + d_max <= 64), and a
// block whose radius breaks that condition flags every query (pass B is exact).
#ifndef AERO_F16_PIPE
#define AERO_F16_PIPE 2
#endif
#ifndef AERO_F16_WPE
#define AERO_F16_WPE 4
#endif
constexpr int kF16QPB = kPassAQPB[kPassAF16s];  // 4 waves x 32 queries x kF16Cols
constexpr int kF16Pipe = AERO_F16_PIPE;          // products reduced together
constexpr float kF16FarT = 32768.0f;
static_assert(kF16Cols % kF16Pipe == 0, "column blocks come in groups of kF16Pipe");
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ void split_half(float v, _Float16& hi, _Float16& lo) {
  hi = (_Float16)v;
  lo = (_Float16)(v - (float)hi);
}

// (at most 512 / AERO_F16_WPE registers: four waves per SIMD by default, where the
// scheduler would otherwise keep four products in flight at three waves)
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(AERO_F16_WPE))) void
k_min_dist_approx_f16s(const QuerySet* __restrict__ sets, int n_sets) {
  __shared__ half8 tile[kTilePts];
  __shared__ float red[7][4];
  const int64_t bid = blockIdx.x;
  const int s = find_owner(sets, n_sets, bid, [](const QuerySet& q) { return q.block_base; });
  const QuerySet S = sets[s];
  const int64_t local = bid - S.block_base;
  const int qb = (int)(local / S.n_chunks), ch = (int)(local % S.n_chunks);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int col = lane & 31, kh = lane >> 5;
  const int64_t slot0 = (int64_t)qb * kF16QPB + w * (32 * kF16Cols) + col;  // + 32 b
  // The block's positions are read twice (bounds, then the split operands), so
  // that only the operands stay in registers.
  unsigned okm = 0;  // bit b: column block b's query of this lane exists
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
#pragma unroll
  for (int b = 0; b < kF16Cols; ++b) {
    const int64_t slot = slot0 + b * 32;
    if (slot < S.Q) {
      okm |= 1u << b;
      const float p[3] = {S.sp[slot], S.sp[S.Q + slot], S.sp[2 * S.Q + slot]};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        lo[a] = fminf(lo[a], p[a]);
        hi[a] = fmaxf(hi[a], p[a]);
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = wave_minf(lo[a]);
    hi[a] = wave_maxf(hi[a]);
  }
  if (lane == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      red[a][w] = lo[a];
      red[3 + a][w] = hi[a];
    }
  }
  __syncthreads();
  float c[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float l = fminf(fminf(red[a][0], red[a][1]), fminf(red[a][2], red[a][3]));
    const float h = fmaxf(fmaxf(red[3 + a][0], red[3 + a][1]), fmaxf(red[3 + a][2], red[3 + a][3]));
    c[a] = 0.5f * l + 0.5f * h;
  }
  half8 bop[kF16Cols];
  float pp[kF16Cols], tmin[kF16Cols], rr = 0.0f;
#pragma unroll
  for (int b = 0; b < kF16Cols; ++b) {
    const bool ok = (okm >> b) & 1u;
    const int64_t qs = ok ? slot0 + b * 32 : 0;  // positions in slot order
    const float x = S.sp[qs] - c[0], y = S.sp[S.Q + qs] - c[1], z = S.sp[2 * S.Q + qs] - c[2];
    pp[b] = fmaf(z, z, fmaf(y, y, x * x));
    if (ok) rr = fmaxf(rr, pp[b]);
    _Float16 xh, xl, yh, yl, zh, zl;
    split_half(x, xh, xl);
    split_half(y, yh, yl);
    split_half(z, zh, zl);
    const _Float16 one = ok ? (_Float16)1.0f : (_Float16)0.0f;
    const _Float16 zero = (_Float16)0.0f;
    half8 v;
    if (kh == 0) {
      v[0] = xh; v[1] = yh; v[2] = zh; v[3] = one;
      v[4] = xh; v[5] = yh; v[6] = zh; v[7] = one;
    } else {
      v[0] = xl; v[1] = yl; v[2] = zl; v[3] = zero;
      v[4] = xl; v[5] = yl; v[6] = zl; v[7] = zero;
    }
    if (!ok) v = (half8){};
    bop[b] = v;
    tmin[b] = kF16FarT;
  }
  rr = wave_maxf(rr);
  if (lane == 0) red[6][w] = rr;
  __syncthreads();
  const float R2 = fmaxf(fmaxf(red[6][0], red[6][1]), fmaxf(red[6][2], red[6][3]));
  const float R = sqrtf(R2) * 1.001f;
  const float span = R + S.d_max;
  const float thr = (span <= 64.0f) ? S.d_max * S.d_max + 0x1p-15f * span * span + 1e-6f
                                    : INFINITY;
  if (tid == 0 && ch == 0) {
    S.thresh[qb] = thr;
    S.seg_count[qb] = 0;
  }
  const floatx16 zacc = {};
  const int64_t g0 = (int64_t)ch * S.chunk_pts;
  const int64_t g1 = min<int64_t>(g0 + S.chunk_pts, S.n_points);
  for (int64_t base = g0; base < g1; base += kTilePts) {
    const int cnt = (int)min<int64_t>(kTilePts, g1 - base);
    const int cnt32 = (cnt + 31) & ~31;  // groups of 32 points, padded
    for (int pt = tid; pt < cnt32; pt += kBlock) {
      const bool in = pt < cnt;
      const int64_t gg = in ? base + pt : base;
      const float ox = S.cloud[3 * gg] - c[0];
      const float oy = S.cloud[3 * gg + 1] - c[1];
      const float oz = S.cloud[3 * gg + 2] - c[2];
      const float n = fmaf(oz, oz, fmaf(oy, oy, ox * ox));
      half8 rec = {};
      if (in && n < 16384.0f) {
        _Float16 xh, xl, yh, yl, zh, zl, nh, nl;
        split_half(-2.0f * ox, xh, xl);
        split_half(-2.0f * oy, yh, yl);
        split_half(-2.0f * oz, zh, zl);
        split_half(n, nh, nl);
        rec[0] = xh; rec[1] = yh; rec[2] = zh; rec[3] = nh;
        rec[4] = xl; rec[5] = yl; rec[6] = zl; rec[7] = nl;
      } else {
        rec[3] = (_Float16)kF16FarT;
      }
      tile[pt] = rec;
    }
    __syncthreads();
    float tt[kF16Cols];
#pragma unroll
    for (int b = 0; b < kF16Cols; ++b) tt[b] = kF16FarT;
    for (int g = 0; g < cnt32; g += 32) {
      const half8 a = tile[g + col];
      // kF16Pipe products in flight: the minima of one overlap the next MFMA
#pragma unroll
      for (int b = 0; b < kF16Cols; b += kF16Pipe) {
        floatx16 dv[kF16Pipe];
#pragma unroll
        for (int j = 0; j < kF16Pipe; ++j)
          dv[j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, bop[b + j], zacc, 0, 0, 0);
#pragma unroll
        for (int j = 0; j < kF16Pipe; ++j) {
          float m = tt[b + j];
#pragma unroll
          for (int r = 0; r < 16; r += 2) m = fminf(fminf(m, dv[j][r]), dv[j][r + 1]);
          tt[b + j] = m;
        }
      }
    }
    bool hit = false;
#pragma unroll
    for (int b = 0; b < kF16Cols; ++b) {
      hit |= ((okm >> b) & 1u) && pp[b] + tt[b] < thr;
      tmin[b] = fminf(tmin[b], tt[b]);
    }
    if (__syncthreads_or(hit) && tid == 0)
      append_block_hits(S, qb, base / kTilePts, red, pass_b_reach2(thr, S.d_max));
  }
#pragma unroll
  for (int b = 0; b < kF16Cols; ++b) {
    float v = tmin[b];
    v = fminf(v, __shfl_xor(v, 32, 64));   // the two lane halves hold different rows
    if (((okm >> b) & 1u) && kh == 0)
      atomicMin(S.out_slot + slot0 + b * 32, __float_as_uint(fmaxf(pp[b] + v, 0.0f)));
  }
}

}  // namespace

hipError_t launch_min_dist_approx_matrix(const QuerySet* d_sets, int n_sets, int64_t total_blocks,
                                         int variant, hipStream_t s) {
  if (total_blocks > 0) {
    if (variant == kPassAF16s)
      k_min_dist_approx_f16s<<<(unsigned)total_blocks, kBlock, 0, s>>>(d_sets, n_sets);
    else
      k_min_dist_approx_mfma<<<(unsigned)total_blocks, kBlock, 0, s>>>(d_sets, n_sets);
  }
  return hipGetLastError();
}

}  // namespace aero
