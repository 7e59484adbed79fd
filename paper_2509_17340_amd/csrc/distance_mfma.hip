// Pass A of the nearest-distance computation on the half-precision matrix cores.
//
// Built with finite-math (every value here is a finite squared distance or a
// finite padding constant), so that chained fminf become v_min3_f32 without
// NaN canonicalisation, and with MFMA results in VGPRs (no accumulator-register
// reads); the compiler inserts the MFMA-to-VALU wait states.  The kernel writes the
// same outputs as the VALU pass A: per item, the hit words of the block's queries
// whose value (exact up to the stated rounding for every pair closer than d_max) came
// under the block's flag bound in the item's sub-tile, and the mark of every item
// with such a query.
//
// Every recentred coordinate is split into two halves, v = hi + lo (hi = half(v),
// lo = half(v - hi)), and one v_mfma_f32_32x32x16_f16 evaluates, for 32 cloud
// points x 32 queries,
//   t = n_hi + n_lo - 2 (o_hi.p_hi + o_lo.p_hi + o_hi.p_lo + o_lo.p_lo)
// with the K = 16 slots laid out as
//   A (point)  [-2o_hi, n_hi, -2o_lo, n_lo | -2o_hi, n_hi, -2o_lo, n_lo]
//   B (query)  [  p_hi,    1,   p_hi,    1 |   p_lo,    0,   p_lo,    0]
// (the zero query slots cancel the repeated norms, so both lane halves read the
// same 16-byte point record from LDS).  Half products are exact in the
// single-precision accumulator, so t carries the split error (2^-22 relative per
// coordinate) plus the accumulation rounding; the cull step's bound for this
// variant is four times the single-precision pass's one.  Halves cover |v| < 65504:
// points with |o'| >= 128 become the constant t = 32768 (never flagged; they are
// provably farther than d_max whenever R + d_max <= 64), and a block whose radius
// breaks that condition has an infinite bound and flags every query (pass B is
// exact).
//
// The kernel runs on a persistent grid over the cull step's item list: workgroup g
// takes the g-th run of ceil(items / grid) consecutive items.  A block's queries are
// set up (positions recentred on the block's centre, split, in registers) when the
// run reaches its first item; each item's 256 points are staged in LDS (double
// buffered: the next item's point is loaded while this one is reduced).  Query
// 32 COLS w + 32 b + col of the block (wave w, column block b, column col) is bit col
// of hit word COLS w + b.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "aero_device.h"
#include "aero_internal.h"

namespace aero {
namespace {

#ifndef AERO_F16_PIPE
#define AERO_F16_PIPE 2
#endif
#ifndef AERO_F16_WPE
#define AERO_F16_WPE 4
#endif
constexpr int kF16Pipe = AERO_F16_PIPE;  // products reduced together
constexpr float kF16FarT = 32768.0f;

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ void split_half(float v, _Float16& hi, _Float16& lo) {
  hi = (_Float16)v;
  lo = (_Float16)(v - (float)hi);
}

// The LDS record of a cloud point recentred on the block centre.
__device__ __forceinline__ half8 point_record(float ox, float oy, float oz, bool in) {
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
  return rec;
}

// (at most 512 / AERO_F16_WPE registers: four waves per SIMD by default)
template <int COLS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(AERO_F16_WPE))) void
k_pass_a_f16s(const QuerySet* __restrict__ sets, int n_sets, const int2* __restrict__ items,
              const int32_t* __restrict__ item_count, unsigned char* __restrict__ hitf) {
  static_assert(COLS % kF16Pipe == 0, "column blocks come in groups of kF16Pipe");
  constexpr int QPB = 4 * 32 * COLS;
  constexpr int W = QPB / 32;  // hit words per item
  __shared__ half8 tile[2][kSubPts];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int col = lane & 31, kh = lane >> 5;
  const int64_t total = *item_count;
  const int64_t G = gridDim.x;
  const int64_t per = (total + G - 1) / G;
  const int64_t i0 = (int64_t)blockIdx.x * per, i1 = min<int64_t>(total, i0 + per);
  if (i0 >= i1) return;  // block-uniform
  SetCache cache{0, 0, 0};
  // the current query block
  int64_t cur = -1;
  unsigned okm = 0;  // bit b: column block b's query of this lane exists
  float c[3] = {0.0f, 0.0f, 0.0f}, thr = 0.0f;
  // the bounding box of this wave's queries and the block's reach: a 32-point group of
  // a sub-tile whose box lies beyond it cannot hold a point whose value falls under
  // the bound, so the wave skips it
  float wlo[3] = {0.0f, 0.0f, 0.0f}, whi[3] = {0.0f, 0.0f, 0.0f}, wlim = 0.0f;
  half8 bop[COLS];
  float pp[COLS];
  int64_t qslot0 = 0;         // this lane's slot of column block 0
  unsigned* amin = nullptr;   // the block's set's least pass-A values
  // each query's least value over the block's items taken so far by this workgroup
  // (they come in runs): one atomic minimum per query and run instead of per item
  float tmin[COLS];
#pragma unroll
  for (int b = 0; b < COLS; ++b) tmin[b] = INFINITY;
  auto flush = [&]() {
    if (kh == 0 && amin) {
#pragma unroll
      for (int b = 0; b < COLS; ++b)
        if (((okm >> b) & 1u) && tmin[b] < thr)  // existing queries that came under
          atomicMin(amin + qslot0 + b * 32, __float_as_uint(fmaxf(tmin[b], 0.0f)));
    }
#pragma unroll
    for (int b = 0; b < COLS; ++b) tmin[b] = INFINITY;
  };
  // the hit words of every set of the call share one array
  AERO_GLOBAL uint32_t* __restrict__ hmask = global_ptr(sets[0].hmask);
  const int64_t mask_items = sets[0].mask_words / W;  // items with room for their words
  // the first item's point
  int2 it = items[i0];
  int ns = set_of(sets, n_sets, it.x, cache);
  float ox, oy, oz;
  int32_t oidx;
  bool oin;
  int cnt;
  item_point(sets[ns], (unsigned)it.y, ox, oy, oz, oidx, oin, cnt);
  bool valid = block_of(sets[ns], it.x) && cnt > 0;
  int buf = 0;
  for (int64_t i = i0; i < i1; ++i) {
    const int64_t gqb = it.x;
    const int icnt = cnt;
    const bool ivalid = valid;
    const unsigned iys = (unsigned)it.y;
    const int ins = ns;
    if (ivalid && gqb != cur) {  // block-uniform
      flush();  // the previous block's least values
      const QuerySet& S = sets[ns];
      const int64_t qb = gqb - S.qb_base;
      const int64_t Q = S.Q;
      const float* __restrict__ sp = S.sp;
      const float4 bi = S.binfo[qb];
      c[0] = bi.x;
      c[1] = bi.y;
      c[2] = bi.z;
      thr = bi.w;
      const int64_t slot0 = qb * QPB + w * (32 * COLS) + col;
      qslot0 = slot0;
      amin = S.amin;
      wlim = S.cull ? reach_limit(thr, S.d_max) : INFINITY;  // brute force: every group
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        wlo[a] = INFINITY;
        whi[a] = -INFINITY;
      }
      okm = 0;
#pragma unroll
      for (int b = 0; b < COLS; ++b) {
        const int64_t slot = slot0 + b * 32;
        const bool ok = slot < Q;
        okm |= ok ? 1u << b : 0u;
        const int64_t qs = ok ? slot : 0;  // positions in slot order
        const float ax = sp[qs], ay = sp[Q + qs], az = sp[2 * Q + qs];
        if (ok) {
          wlo[0] = fminf(wlo[0], ax);
          wlo[1] = fminf(wlo[1], ay);
          wlo[2] = fminf(wlo[2], az);
          whi[0] = fmaxf(whi[0], ax);
          whi[1] = fmaxf(whi[1], ay);
          whi[2] = fmaxf(whi[2], az);
        }
        const float x = ax - c[0], y = ay - c[1], z = az - c[2];
        pp[b] = fmaf(z, z, fmaf(y, y, x * x));
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
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        wlo[a] = wave_minf(wlo[a]);
        whi[a] = wave_maxf(whi[a]);
      }
      cur = gqb;
    }
    if (ivalid) tile[buf][tid] = point_record(ox - c[0], oy - c[1], oz - c[2], oin);
    // the next item's point, loaded while this one is reduced
    if (i + 1 < i1) {
      it = items[i + 1];
      ns = set_of(sets, n_sets, it.x, cache);
      item_point(sets[ns], (unsigned)it.y, ox, oy, oz, oidx, oin, cnt);
      valid = block_of(sets[ns], it.x) && cnt > 0;
    }
    if (!ivalid) continue;  // block-uniform; the buffers alternate over processed items only
    __syncthreads();
    const half8* tl = tile[buf];
    buf ^= 1;
    float tt[COLS];
#pragma unroll
    for (int b = 0; b < COLS; ++b) tt[b] = kF16FarT;
    // the item's 32-point groups within reach of this wave's queries (lane q tests
    // group q; bit q of the ballot)
    const QuerySet& IS = sets[ins];
    const float* gbs = ((iys >> 31) && IS.scloud ? IS.sgbox : IS.gbox) +
                       6 * (int64_t)(iys & 0x7fffffffu) * kGroupsPerSub;
    const uint64_t keep = __ballot(lane < kGroupsPerSub && lane * 32 < icnt &&
                                   box_dist2(gbs + 6 * min(lane, kGroupsPerSub - 1), wlo, whi) <=
                                       wlim);
    // the groups taken, in order (only groups with points can be set: lane * 32 <
    // icnt), each one's point record read from LDS while the previous one's products
    // are reduced
    uint32_t left = (uint32_t)keep;
    half8 a_next = {};
    if (left) a_next = tl[32 * (__ffs(left) - 1) + col];
    while (left) {  // wave-uniform
      const half8 a = a_next;
      left &= left - 1u;
      if (left) a_next = tl[32 * (__ffs(left) - 1) + col];
      // kF16Pipe products in flight: the minima of one overlap the next MFMA
#pragma unroll
      for (int b = 0; b < COLS; b += kF16Pipe) {
        floatx16 dv[kF16Pipe];
#pragma unroll
        for (int j = 0; j < kF16Pipe; ++j)
          dv[j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, bop[b + j], (floatx16){}, 0, 0, 0);
#pragma unroll
        for (int j = 0; j < kF16Pipe; ++j) {
          // a tree of minima (depth 3, eight min3) rather than a chain of eight
          const floatx16& d = dv[j];
          const float t0 = fminf(fminf(d[0], d[1]), d[2]), t1 = fminf(fminf(d[3], d[4]), d[5]);
          const float t2 = fminf(fminf(d[6], d[7]), d[8]), t3 = fminf(fminf(d[9], d[10]), d[11]);
          const float t4 = fminf(fminf(d[12], d[13]), d[14]);
          const float u0 = fminf(fminf(t0, t1), t2), u1 = fminf(fminf(t3, t4), d[15]);
          tt[b + j] = fminf(fminf(tt[b + j], u0), u1);
        }
      }
    }
    bool hit = false;
    const bool room = i < mask_items;  // block-uniform
#pragma unroll
    for (int b = 0; b < COLS; ++b) {
      // the two lane halves hold different rows (points) of the same column (query):
      // one lane-half swap gives every lane both halves' minima
      const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(tt[b]),
                                                       __float_as_uint(tt[b]), false, false);
      const float v = fminf(__uint_as_float(sw[0]), __uint_as_float(sw[1]));
      const float t = pp[b] + v;
      const bool hq = ((okm >> b) & 1u) && t < thr;
      hit |= hq;
      const uint64_t hb = __ballot(hq);
      if (room && lane == 0) hmask[i * W + w * COLS + b] = (uint32_t)(hb & 0xffffffffull);
      tmin[b] = fminf(tmin[b], t);  // both lane halves hold it: the lower one stores
    }
    mark_hit(hit, hitf, i);
  }
  flush();
}

// The pairs pass A evaluates, for the statistics call: the same 32-point groups each
// wave takes (the matrix-core variants skip the groups beyond reach of the wave's
// positions; the VALU variant takes every group).  pass_a_pairs[0] sums existing
// positions x points of the groups taken, pass_a_pairs[1] the matrix-core products'
// pairs (32 points x the wave's 32 COLS columns per group taken, padding included).
__device__ unsigned long long pass_a_pairs[2];
__global__ __launch_bounds__(kBlock) void k_pass_a_count(const QuerySet* __restrict__ sets,
                                                         int n_sets,
                                                         const int2* __restrict__ items,
                                                         const int32_t* __restrict__ item_count) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t total = *item_count;
  SetCache cache{0, 0, 0};
  unsigned long long ev = 0, pr = 0;  // this wave's sums (lane 0)
  for (int64_t i = blockIdx.x; i < total; i += gridDim.x) {
    const int2 it = items[i];
    const QuerySet& S = sets[set_of(sets, n_sets, it.x, cache)];
    if (!block_of(S, it.x) || S.n_points <= 0) continue;
    const unsigned ys = (unsigned)it.y;
    const int64_t g0 = (int64_t)(ys & 0x7fffffffu) * kSubPts;
    const bool srt = (ys >> 31) != 0;
    const int cnt = (g0 < S.n_points && (!srt || S.scloud))
                        ? (int)min<int64_t>(kSubPts, S.n_points - g0)
                        : 0;
    if (cnt <= 0) continue;
    const int64_t qb = it.x - S.qb_base, Q = S.Q;
    const int qpb = S.qpbA;
    if (qpb == kQueriesPerBlock) {  // the VALU pass: every group of the item
      if (threadIdx.x == 0) {
        const int64_t nq = min<int64_t>(qpb, Q - qb * qpb);
        ev += nq * cnt;
        pr += nq * cnt;
      }
      continue;
    }
    const int per_w = qpb / 4;  // 32 COLS positions per wave
    const int64_t s0 = qb * qpb + (int64_t)w * per_w;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int j = lane; j < per_w; j += 64) {
      const int64_t q = s0 + j;
      if (q >= Q) break;
      const float p[3] = {S.sp[q], S.sp[Q + q], S.sp[2 * Q + q]};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        lo[a] = fminf(lo[a], p[a]);
        hi[a] = fmaxf(hi[a], p[a]);
      }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = wave_minf(lo[a]);
      hi[a] = wave_maxf(hi[a]);
    }
    const int64_t nqw = max<int64_t>(0, min<int64_t>(per_w, Q - s0));
    const float wlim = S.cull ? reach_limit(S.binfo[qb].w, S.d_max) : INFINITY;
    const float* gbs = (srt && S.scloud ? S.sgbox : S.gbox) +
                       6 * (int64_t)(ys & 0x7fffffffu) * kGroupsPerSub;
    const uint64_t keep = __ballot(lane < kGroupsPerSub && lane * 32 < cnt &&
                                   box_dist2(gbs + 6 * min(lane, kGroupsPerSub - 1), lo, hi) <=
                                       wlim);
    if (lane == 0)
      for (int g = 0; g < kGroupsPerSub; ++g)
        if ((keep >> g) & 1ull) {
          ev += (unsigned long long)(nqw * min(32, cnt - 32 * g));
          pr += (unsigned long long)(32 * per_w);
        }
  }
  if (lane == 0) {
    atomicAdd(&pass_a_pairs[0], ev);
    atomicAdd(&pass_a_pairs[1], pr);
  }
}

}  // namespace

hipError_t count_pass_a_pairs(const QuerySet* d_sets, int n_sets, const int2* items,
                              const int32_t* item_count, int64_t max_items,
                              unsigned long long* h_pairs) {
  const unsigned long long zero[2] = {0, 0};
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(pass_a_pairs), zero, sizeof zero, 0,
                                   hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  if (max_items > 0) {
    const unsigned grid = (unsigned)(max_items < 4096 ? max_items : 4096);
    k_pass_a_count<<<grid, kBlock, 0, 0>>>(d_sets, n_sets, items, item_count);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = hipDeviceSynchronize()) != hipSuccess) return e;
  return hipMemcpyFromSymbol(h_pairs, HIP_SYMBOL(pass_a_pairs), sizeof zero, 0,
                             hipMemcpyDeviceToHost);
}

hipError_t launch_pass_a_matrix(const QuerySet* d_sets, int n_sets, const int2* items,
                                const int32_t* item_count, unsigned char* hitf, int64_t max_items,
                                int variant, int grid_max, hipStream_t s) {
  if (max_items > 0) {
    // persistent workgroups (the autotuner's choice), each over a range of items
    const unsigned grid = (unsigned)(max_items < grid_max ? max_items : grid_max);
    if (variant == kPassAF16s4)
      k_pass_a_f16s<4><<<grid, kBlock, 0, s>>>(d_sets, n_sets, items, item_count, hitf);
    else
      k_pass_a_f16s<8><<<grid, kBlock, 0, s>>>(d_sets, n_sets, items, item_count, hitf);
  }
  return hipGetLastError();
}

}  // namespace aero
