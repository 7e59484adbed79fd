// Cull step of the nearest-distance computation (the d_t of the collision cost,
// Sec. IV-C): which cloud sub-tiles each query block of the first pass must visit.
//
// The collision penalty vanishes from d_max on, so a query block only needs the
// cloud points within d_max of its queries (plus those whose first-pass value could
// fall under the block's flag bound, all within the reach sqrt(2 thresh - d_max^2)).
// The cloud is cut into tiles of kTilePts and sub-tiles of kSubPts consecutive
// points with bounding boxes, and runs of kSuperTiles tiles (super-tiles) with theirs;
// a block lists every sub-tile whose box lies within reach of the block's box,
// testing super-tiles, then their tiles, then the tiles' sub-tiles (each box contains
// the boxes below it).  Two orders of the cloud are considered when the cloud has
// been spatially sorted: the order it was given in (a LiDAR sweep in beam order is
// already made of compact runs) and the Morton order; each block takes the one that
// lists fewer sub-tiles.  A block's items are written consecutively, so that the
// first pass sets a block up once per run of its items.
//
//   k_sorted_boxes  tile and sub-tile boxes of the sorted clouds
//   k_super_boxes   boxes of kSuperTiles consecutive tiles, both orders
//   k_cull          per query block: bounding box, centre, radius, flag bound,
//                   and its items
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "aero_device.h"
#include "aero_internal.h"

namespace aero {
namespace {

__global__ __launch_bounds__(kBlock) void k_sorted_boxes(const QuerySet* __restrict__ sets,
                                                         int n_sets) {
  const int64_t t = blockIdx.x;
  const int s = find_owner(sets, n_sets, t, [](const QuerySet& q) { return q.tile_base; });
  const QuerySet& S = sets[s];
  if (!S.scloud) return;  // block-uniform
  tile_boxes(nullptr, S.scloud, S.n_points, t - S.tile_base, S.stbox, S.ssbox, S.sgbox);
}

// One workgroup per set: the super-tile boxes of the raw cloud and, when sorted, of
// the sorted cloud, from their tile boxes.
__global__ __launch_bounds__(kBlock) void k_super_boxes(const QuerySet* __restrict__ sets) {
  const QuerySet& S = sets[blockIdx.x];
  if (S.n_qblocks <= 0 || !S.tbox) return;  // block-uniform: a two-pass set only
  const int64_t n_tiles = S.n_tiles;
  const int64_t n_super = (n_tiles + kSuperTiles - 1) / kSuperTiles;
  for (int64_t i = threadIdx.x; i < 2 * n_super; i += kBlock) {
    const int order = i >= n_super ? 1 : 0;
    const int64_t u = i - order * n_super;
    const float* __restrict__ tb = order ? S.stbox : S.tbox;
    float* __restrict__ ub = order ? S.subox : S.ubox;
    if (!tb || !ub) continue;
    float b[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    const int64_t t1 = min<int64_t>(n_tiles, (u + 1) * kSuperTiles);
    for (int64_t t = u * kSuperTiles; t < t1; ++t) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        b[a] = fminf(b[a], tb[6 * t + a]);
        b[3 + a] = fmaxf(b[3 + a], tb[6 * t + 3 + a]);
      }
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) ub[6 * u + a] = b[a];
  }
}

__device__ inline int wave_sum_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sub-tiles of one cloud order within reach of the block box [lo, hi]: bit j of the
// result is sub-tile 4 t + j of tile t.  The sub-tile boxes are read together with
// the tile's (one memory round trip instead of two).
__device__ inline unsigned reach_mask(const float* __restrict__ tbox,
                                      const float* __restrict__ sbox, int64_t t, int64_t n_sub,
                                      const float lo[3], const float hi[3], float lim) {
  float tb[6], sb[kTileSplit][6];
#pragma unroll
  for (int a = 0; a < 6; ++a) tb[a] = tbox[6 * t + a];
#pragma unroll
  for (int j = 0; j < kTileSplit; ++j) {
    const int64_t sub = min<int64_t>(t * kTileSplit + j, n_sub - 1);
#pragma unroll
    for (int a = 0; a < 6; ++a) sb[j][a] = sbox[6 * sub + a];
  }
  unsigned mask = 0;
  if (box_dist2(tb, lo, hi) <= lim) {
#pragma unroll
    for (int j = 0; j < kTileSplit; ++j) {
      const int64_t sub = t * kTileSplit + j;
      if (sub < n_sub && box_dist2(sb[j], lo, hi) <= lim) mask |= 1u << j;
    }
  }
  return mask;
}

// Calls f(t, mask) for every tile t of one cloud order whose super-tile lies within
// reach of the block box, with the reach mask of its sub-tiles, the tiles in
// increasing order across the wave's lanes (16 lanes per super-tile, four super-
// tiles per round).  Every lane calls f the same number of times, with t = -1 and
// mask 0 where it holds no tile, so that f may scan over the wave.
template <typename F>
__device__ inline void scan_reach(const float* __restrict__ ub, const float* __restrict__ tbox,
                                  const float* __restrict__ sbox, int64_t n_tiles,
                                  int64_t n_sub, const float lo[3], const float hi[3],
                                  float lim, int lane, F&& f) {
  static_assert(kSuperTiles == 16, "four super-tiles of 16 tiles per wave round");
  const int64_t n_super = (n_tiles + kSuperTiles - 1) / kSuperTiles;
  for (int64_t u0 = 0; u0 < n_super; u0 += 64) {
    const int64_t u = u0 + lane;
    const bool near = u < n_super && box_dist2(ub + 6 * u, lo, hi) <= lim;
    unsigned long long hits = __ballot(near);
    while (hits) {  // wave-uniform
      int take[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        take[i] = hits ? __ffsll((long long)hits) - 1 : -1;
        hits &= hits - 1ull;
      }
      const int mine = take[lane >> 4];
      const int64_t t = mine >= 0 ? (u0 + mine) * kSuperTiles + (lane & 15) : n_tiles;
      const unsigned mask = t < n_tiles ? reach_mask(tbox, sbox, t, n_sub, lo, hi, lim) : 0u;
      f(t < n_tiles ? t : (int64_t)-1, mask);
    }
  }
}

// One wave per query block, kCullWaves per workgroup.  The waves' item counts meet in
// LDS and the workgroup takes its run of the item list with one atomic addition (one
// per wave put every wave of the grid in line on a single counter).
#ifndef AERO_CULL_WAVES
#define AERO_CULL_WAVES 4
#endif
constexpr int kCullWaves = AERO_CULL_WAVES;
__global__ __launch_bounds__(64 * kCullWaves) void k_cull(const QuerySet* __restrict__ sets,
                                                          int n_sets, int64_t total_qblocks,
                                                          int variant) {
  __shared__ int wstart[kCullWaves];  // each wave's count, then its offset in the run
  __shared__ int wgbase;              // the workgroup's run in the item list
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t gqb0 = (int64_t)blockIdx.x * kCullWaves + w;
  const bool live = gqb0 < total_qblocks;  // wave-uniform
  const int64_t gqb = live ? gqb0 : total_qblocks - 1;  // a valid block for the others
  const int s = find_owner(sets, n_sets, gqb, [](const QuerySet& q) { return q.qb_base; });
  const QuerySet& S = sets[s];
  const int64_t qb = gqb - S.qb_base;
  const int64_t Q = S.Q;
  const float* __restrict__ sp = S.sp;
  const int64_t s0 = qb * S.qpbA, s1 = min<int64_t>(Q, s0 + S.qpbA);
  // bounding box of the block's positions (exact min/max: order independent); the
  // positions are read kCullU per lane at a time, lanes past the block's end taking
  // its first position again
  constexpr int kCullU = 8;
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i0 = s0 + lane; i0 < s1; i0 += 64 * kCullU) {
    float p[kCullU][3];
#pragma unroll
    for (int u = 0; u < kCullU; ++u) {
      const int64_t i = i0 + 64 * u < s1 ? i0 + 64 * u : s0;
      p[u][0] = sp[i];
      p[u][1] = sp[Q + i];
      p[u][2] = sp[2 * Q + i];
    }
#pragma unroll
    for (int u = 0; u < kCullU; ++u)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        lo[a] = fminf(lo[a], p[u][a]);
        hi[a] = fmaxf(hi[a], p[u][a]);
      }
  }
  float c[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = wave_minf(lo[a]);
    hi[a] = wave_maxf(hi[a]);
    c[a] = 0.5f * lo[a] + 0.5f * hi[a];
  }
  // radius about the centre, formed as the first pass forms |p'|^2
  float rr = 0.0f;
  for (int64_t i0 = s0 + lane; i0 < s1; i0 += 64 * kCullU) {
    float p[kCullU][3];
#pragma unroll
    for (int u = 0; u < kCullU; ++u) {
      const int64_t i = i0 + 64 * u < s1 ? i0 + 64 * u : s0;
      p[u][0] = sp[i];
      p[u][1] = sp[Q + i];
      p[u][2] = sp[2 * Q + i];
    }
#pragma unroll
    for (int u = 0; u < kCullU; ++u) {
      const float x = p[u][0] - c[0], y = p[u][1] - c[1], z = p[u][2] - c[2];
      rr = fmaxf(rr, fmaf(z, z, fmaf(y, y, x * x)));
    }
  }
  rr = wave_maxf(rr);
  // Flag bound: the pass-A value of a pair within d_max errs by at most
  //   VALU  about 26 u (R + d_max)^2 with u = 2^-24 (three FMAs on recentred
  //         coordinates): 2^-17 (R + d_max)^2 leaves a 5x margin;
  //   split FP16 matrix cores  2^-15 (R + d_max)^2, valid while the recentred
  //         coordinates fit the halves (R + d_max <= 64); a wider block flags all.
  const float d_max = S.d_max;
  float thr;
  if (variant == kPassAValu) {
    const float span = sqrtf(rr) * 1.001f + d_max;
    thr = d_max * d_max + 0x1p-17f * span * span + 1e-6f;
  } else {
    const float span = sqrtf(rr) * 1.001f + d_max;
    thr = span <= 64.0f ? d_max * d_max + 0x1p-15f * span * span + 1e-6f : INFINITY;
  }
  if (live && lane == 0) S.binfo[qb] = make_float4(c[0], c[1], c[2], thr);
  const int64_t n_tiles = S.n_tiles;
  const int64_t n_sub = ((int64_t)S.n_points + kSubPts - 1) / kSubPts;
  const float lim = S.cull ? reach_limit(thr, d_max) : INFINITY;
  // items of each order
  int cnt_raw = 0, cnt_srt = 0;
  scan_reach(S.ubox, S.tbox, S.sbox, n_tiles, n_sub, lo, hi, lim, lane,
             [&](int64_t, unsigned mask) { cnt_raw += __popc(mask); });
  cnt_raw = wave_sum_i(cnt_raw);
  const bool sorted_ok = S.scloud != nullptr && S.cull;
  if (sorted_ok) {
    scan_reach(S.subox, S.stbox, S.ssbox, n_tiles, n_sub, lo, hi, lim, lane,
               [&](int64_t, unsigned mask) { cnt_srt += __popc(mask); });
    cnt_srt = wave_sum_i(cnt_srt);
  }
  const int order = (sorted_ok && cnt_srt < cnt_raw) ? 1 : 0;
  const int cnt = live ? (order ? cnt_srt : cnt_raw) : 0;
  if (lane == 0) wstart[w] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int v = 0; v < kCullWaves; ++v) {
      const int cv = wstart[v];
      wstart[v] = tot;
      tot += cv;
    }
    // wave 0 is live whenever any wave is, and every set of the call shares the counter
    wgbase = tot > 0 ? atomicAdd(S.item_count, tot) : 0;
  }
  __syncthreads();
  if (cnt == 0) return;  // wave-uniform; no barrier follows
  const int base = wgbase + wstart[w];
  const float* __restrict__ ub = order ? S.subox : S.ubox;
  const float* __restrict__ tb = order ? S.stbox : S.tbox;
  const float* __restrict__ sb = order ? S.ssbox : S.sbox;
  int2* __restrict__ items = S.items;
  AERO_GLOBAL unsigned char* __restrict__ hitf = global_ptr(S.hitf);
  const unsigned flag = (unsigned)order << 31;
  // the same tests again, now writing the listed sub-tiles in increasing order
  int run = 0;
  scan_reach(ub, tb, sb, n_tiles, n_sub, lo, hi, lim, lane, [&](int64_t t, unsigned mask) {
    const int m = __popc(mask);
    int x = m;  // inclusive scan over the wave
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    int at = base + run + x - m;
#pragma unroll
    for (int j = 0; j < kTileSplit; ++j)
      if ((mask >> j) & 1u) {
        if (at < base + cnt) {  // always, for the same tests; never write past the run
          items[at] = make_int2((int)gqb, (int)((unsigned)(t * kTileSplit + j) | flag));
          hitf[at] = 0;
        }
        ++at;
      }
    run += __shfl(x, 63, 64);
  });
}

}  // namespace

hipError_t launch_sorted_boxes(const QuerySet* d_sets, int n_sets, int64_t total_tiles,
                               hipStream_t s) {
  if (total_tiles > 0) k_sorted_boxes<<<(unsigned)total_tiles, kBlock, 0, s>>>(d_sets, n_sets);
  return hipGetLastError();
}

hipError_t launch_cull(const QuerySet* d_sets, int n_sets, int64_t total_qblocks, int variant,
                       hipStream_t s) {
  if (total_qblocks > 0) {
    k_super_boxes<<<(unsigned)n_sets, kBlock, 0, s>>>(d_sets);
    k_cull<<<(unsigned)((total_qblocks + kCullWaves - 1) / kCullWaves), 64 * kCullWaves, 0, s>>>(
        d_sets, n_sets, total_qblocks, variant);
  }
  return hipGetLastError();
}

}  // namespace aero
