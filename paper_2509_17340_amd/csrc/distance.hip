// Brute-force nearest squared distance from rollout positions to the raw cloud
// (the d_t of the collision cost, Sec. IV-C).
//
//   k_min_dist_exact   direct form (p - o)^2 per pair; cloud tiles staged in LDS
//                      and read as wave-wide broadcasts, kQueriesPerLane queries
//                      per lane in registers.  Over every query of a set, or (pass
//                      B) over a flagged list with a persistent grid.
//   k_min_dist_approx  pass A: the expanded form |o'|^2 - 2 p'.o' with query and
//                      cloud recentred on the query block's bounding-box centre:
//                      three FMAs and half a min3 per pair.  Also writes, per query
//                      block, the bound below which the approximate value may hide
//                      a true distance under d_max (from its rounding-error bound).
//   k_flag             compacts the queries under that bound into a list and resets
//                      them for pass B.
//
// Chunks of the cloud combine through atomicMin on the float bit patterns of the
// non-negative squared distances (exact and order independent), so every result
// is bitwise reproducible.  Queries left unflagged keep their pass-A value, which
// is then provably >= d_max^2: there the collision penalty is 0 whatever the exact
// distance.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "aero_device.h"
#include "aero_internal.h"

namespace aero {
namespace {

constexpr unsigned kInfBits = 0x7f800000u;
constexpr float kFar = 1.0e18f;  // padding point of the direct form: d^2 stays finite
constexpr float kFarT = 1.0e30f;  // padding of the expanded form
constexpr int kPersistBlocks = 2048;

// min(a, b, c) as one VALU instruction (the compiler otherwise pairs two mins).
__device__ __forceinline__ float min3f(float a, float b, float c) {
  float r;
  asm("v_min3_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// Direct-form min over the cloud points [g0, g1) for R queries per lane; with
// kIdx also the lowest point index attaining it (points are visited in
// increasing index order within a lane and ties never replace).
template <int R, bool kIdx>
__device__ inline void direct_range(const QuerySet& S, int64_t g0, int64_t g1, float4* tile,
                                    const float* px, const float* py, const float* pz,
                                    float* best, int32_t* bidx) {
  const int tid = threadIdx.x;
  for (int64_t base = g0; base < g1; base += kTilePts) {
    const int cnt = (int)min<int64_t>(kTilePts, g1 - base);
    const int cnt2 = (cnt + 1) & ~1;  // even: the loop takes points in pairs
    for (int pt = tid; pt < cnt2; pt += kBlock) {
      const int64_t g = base + pt;
      const bool in = pt < cnt;
      const int64_t gg = in ? g : base;  // always a valid address
      const float x = S.cloud[3 * gg], y = S.cloud[3 * gg + 1], z = S.cloud[3 * gg + 2];
      tile[pt] = in ? make_float4(x, y, z, 0.0f) : make_float4(kFar, kFar, kFar, 0.0f);
    }
    __syncthreads();
#pragma unroll 2
    for (int j = 0; j < cnt2; j += 2) {
      const float4 a = tile[j];
      const float4 c = tile[j + 1];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const float ax = px[r] - a.x, ay = py[r] - a.y, az = pz[r] - a.z;
        const float cx = px[r] - c.x, cy = py[r] - c.y, cz = pz[r] - c.z;
        const float da = fmaf(az, az, fmaf(ay, ay, ax * ax));
        const float dc = fmaf(cz, cz, fmaf(cy, cy, cx * cx));
        if constexpr (kIdx) {
          const int ia = (int)(base + j);
          if (da < best[r]) {
            best[r] = da;
            bidx[r] = ia;
          }
          if (dc < best[r]) {
            best[r] = dc;
            bidx[r] = ia + 1;
          }
        } else {
          best[r] = min3f(best[r], da, dc);
        }
      }
    }
    __syncthreads();
  }
}

// Every query of an exact set.  Block = (query block of R * kBlock queries, cloud
// chunk); R (queries per lane) is sized to the set, so that small sets leave few
// lanes idle.
template <int R>
__device__ inline void exact_block(const QuerySet& S, int qb, int ch, float4* tile) {
  const int tid = threadIdx.x;
  float px[R], py[R], pz[R], best[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t q = (int64_t)qb * (R * kBlock) + r * kBlock + tid;
    const int64_t qq = q < S.Q ? q : 0;  // out-of-range lanes read query 0, never stored
    px[r] = S.px[qq];
    py[r] = S.py[qq];
    pz[r] = S.pz[qq];
    best[r] = __uint_as_float(kInfBits);
  }
  const int64_t g0 = (int64_t)ch * S.chunk_pts;
  const int64_t g1 = min<int64_t>(g0 + S.chunk_pts, S.n_points);
  direct_range<R, false>(S, g0, g1, tile, px, py, pz, best, nullptr);
  unsigned* out = S.out + (int64_t)(blockIdx.x % max(S.n_copies, 1)) * S.Q;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t q = (int64_t)qb * (R * kBlock) + r * kBlock + tid;
    if (q < S.Q) atomicMin(out + q, __float_as_uint(best[r]));
  }
}

__global__ __launch_bounds__(kBlock) void k_min_dist_exact(const QuerySet* __restrict__ sets,
                                                           int n_sets) {
  __shared__ float4 tile[kTilePts];
  const int64_t bid = blockIdx.x;
  const int s = find_owner(sets, n_sets, bid, [](const QuerySet& q) { return q.block_base; });
  const QuerySet S = sets[s];
  const int64_t local = bid - S.block_base;
  const int qb = (int)(local / S.n_chunks), ch = (int)(local % S.n_chunks);
  switch (S.qpbA / kBlock) {  // block-uniform
    case 1: exact_block<1>(S, qb, ch, tile); break;
    case 2: exact_block<2>(S, qb, ch, tile); break;
    case 4: exact_block<4>(S, qb, ch, tile); break;
    default: exact_block<kQueriesPerLane>(S, qb, ch, tile); break;
  }
}


// One pass-B item: the flagged queries of query block qb (R per lane; their
// positions as the flag kernel wrote them) against the cloud sub-tile [g0, g1).
// With kIdx also the lowest point index attaining the minimum (points are visited
// in increasing index order and ties never replace).
template <int R, bool kIdx>
__device__ inline void listed_item(const QuerySet& S, int64_t qb, int cnt, int64_t g0, int64_t g1,
                                   float4* tile) {
  const int tid = threadIdx.x;
  const int64_t lbase = qb * S.qpbA;
  float px[R], py[R], pz[R], best[R];
  int32_t qi[R], bidx[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = r * kBlock + tid;
    const bool ok = j < cnt;
    const int64_t e = lbase + (ok ? j : 0);  // cnt >= 1: entry 0 exists
    qi[r] = ok ? S.list[e] : -1;
    const float4 p = S.fpos[e];
    px[r] = p.x;
    py[r] = p.y;
    pz[r] = p.z;
    best[r] = __uint_as_float(kInfBits);
    bidx[r] = 0x7fffffff;
  }
  const int n = (int)(g1 - g0);  // <= kSubPts
  const int n2 = (n + 1) & ~1;    // even: the loop takes points in pairs
  for (int pt = tid; pt < n2; pt += kBlock) {
    const int64_t g = g0 + (pt < n ? pt : 0);  // always a valid address
    tile[pt] = pt < n ? make_float4(S.cloud[3 * g], S.cloud[3 * g + 1], S.cloud[3 * g + 2], 0.0f)
                      : make_float4(kFar, kFar, kFar, 0.0f);
  }
  __syncthreads();
#pragma unroll 2
  for (int j = 0; j < n2; j += 2) {
    const float4 a = tile[j];
    const float4 c = tile[j + 1];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float ax = px[r] - a.x, ay = py[r] - a.y, az = pz[r] - a.z;
      const float cx = px[r] - c.x, cy = py[r] - c.y, cz = pz[r] - c.z;
      const float da = fmaf(az, az, fmaf(ay, ay, ax * ax));
      const float dc = fmaf(cz, cz, fmaf(cy, cy, cx * cx));
      if constexpr (kIdx) {
        const int ia = (int)(g0 + j);
        if (da < best[r]) {
          best[r] = da;
          bidx[r] = ia;
        }
        if (dc < best[r]) {
          best[r] = dc;
          bidx[r] = ia + 1;
        }
      } else {
        best[r] = min3f(best[r], da, dc);
      }
    }
  }
  __syncthreads();  // the next item stages over the tile
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (qi[r] < 0) continue;
    atomicMin(S.out_slot + qi[r], __float_as_uint(best[r]));
    if constexpr (kIdx)
      atomicMin(S.nn + lbase + r * kBlock + tid,
                ((unsigned long long)__float_as_uint(best[r]) << 32) |
                    (unsigned long long)(unsigned)bidx[r]);
  }
}

template <int R>
__device__ inline void listed_item_r(const QuerySet& S, int64_t qb, int cnt, int64_t g0,
                                     int64_t g1, float4* tile) {
  if (S.nn)
    listed_item<R, true>(S, qb, cnt, g0, g1, tile);
  else
    listed_item<R, false>(S, qb, cnt, g0, g1, tile);
}

// Pass B: exact direct form for the flagged queries, only against the sub-tiles that
// pass A listed for their block (a query's nearest point within d_max always lies
// in one).  Persistent grid over the work lists of every two-pass set (each entry
// expanded into its kTileSplit sub-tiles, unlisted ones skipped); the lengths are
// read on the device.
__global__ __launch_bounds__(kBlock) void k_min_dist_listed(const QuerySet* __restrict__ sets,
                                                            int n_sets) {
  __shared__ float4 tile[kSubPts];
  int64_t item_base = 0;
  for (int s = 0; s < n_sets; ++s) {
    const QuerySet& Sref = sets[s];
    if (!Sref.list || Sref.n_points <= 0) continue;
    const int64_t items = (int64_t)*Sref.work_count * kTileSplit;
    int64_t first = ((int64_t)blockIdx.x - item_base) % gridDim.x;
    if (first < 0) first += gridDim.x;
    if (items > 0) {
      const QuerySet S = Sref;
      for (int64_t it = first; it < items; it += gridDim.x) {
        const int2 wk = S.work[it / kTileSplit];
        const int j = (int)(it % kTileSplit);
        if (!((wk.y >> j) & 1)) continue;  // sub-tile not listed
        const int64_t qb = wk.x;
        const int cnt = min(S.seg_count[qb], S.qpbA);
        const int64_t g0 = ((int64_t)((unsigned)wk.y >> 4) * kTileSplit + j) * kSubPts;
        const int64_t g1 = min<int64_t>(g0 + kSubPts, S.n_points);
        if (cnt <= 0 || g0 >= g1) continue;
        const int nr = (cnt + kBlock - 1) / kBlock;
        // exactly as many flagged queries per lane as the block has (no idle groups)
        switch (nr) {
          case 1: listed_item_r<1>(S, qb, cnt, g0, g1, tile); break;
          case 2: listed_item_r<2>(S, qb, cnt, g0, g1, tile); break;
          case 3: listed_item_r<3>(S, qb, cnt, g0, g1, tile); break;
          case 4: listed_item_r<4>(S, qb, cnt, g0, g1, tile); break;
          case 5: listed_item_r<5>(S, qb, cnt, g0, g1, tile); break;
          case 6: listed_item_r<6>(S, qb, cnt, g0, g1, tile); break;
          case 7: listed_item_r<7>(S, qb, cnt, g0, g1, tile); break;
          default: listed_item_r<kQueriesPerLane>(S, qb, cnt, g0, g1, tile); break;
        }
      }
    }
    item_base += items;
  }
}

// Pass A.  Block = (query block, cloud chunk) of a two-pass set.
__global__ __launch_bounds__(kBlock) void k_min_dist_approx(const QuerySet* __restrict__ sets,
                                                            int n_sets) {
  __shared__ float4 tile[kTilePts];
  __shared__ float red[7][4];
  const int64_t bid = blockIdx.x;
  const int s = find_owner(sets, n_sets, bid, [](const QuerySet& q) { return q.block_base; });
  const QuerySet S = sets[s];
  const int64_t local = bid - S.block_base;
  const int qb = (int)(local / S.n_chunks), ch = (int)(local % S.n_chunks);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  constexpr int R = kQueriesPerLane;
  float px[R], py[R], pz[R];
  bool ok[R];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t slot = (int64_t)qb * kQueriesPerBlock + r * kBlock + tid;
    ok[r] = slot < S.Q;
    const int64_t qs = ok[r] ? slot : 0;  // positions in slot order
    px[r] = S.sp[qs];
    py[r] = S.sp[S.Q + qs];
    pz[r] = S.sp[2 * S.Q + qs];
    if (ok[r]) {
      lo[0] = fminf(lo[0], px[r]);
      lo[1] = fminf(lo[1], py[r]);
      lo[2] = fminf(lo[2], pz[r]);
      hi[0] = fmaxf(hi[0], px[r]);
      hi[1] = fmaxf(hi[1], py[r]);
      hi[2] = fmaxf(hi[2], pz[r]);
    }
  }
  // Bounding-box centre of the block's queries (exact min/max, order independent).
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
  float pp[R], tmin[R], rr = 0.0f;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    px[r] -= c[0];
    py[r] -= c[1];
    pz[r] -= c[2];
    pp[r] = fmaf(pz[r], pz[r], fmaf(py[r], py[r], px[r] * px[r]));
    if (ok[r]) rr = fmaxf(rr, pp[r]);
    tmin[r] = kFarT;
  }
  // Rounding-error bound of the pass-A value of any pair within d_max:
  // about 26 u (R + d_max)^2 with u = 2^-24; flag with a 5x margin.
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
  const int64_t g0 = (int64_t)ch * S.chunk_pts;
  const int64_t g1 = min<int64_t>(g0 + S.chunk_pts, S.n_points);
  for (int64_t base = g0; base < g1; base += kTilePts) {
    const int cnt = (int)min<int64_t>(kTilePts, g1 - base);
    const int cnt2 = (cnt + 1) & ~1;
    for (int pt = tid; pt < cnt2; pt += kBlock) {
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
    float tt[R];
#pragma unroll
    for (int r = 0; r < R; ++r) tt[r] = kFarT;
#pragma unroll 4
    for (int j = 0; j < cnt2; j += 2) {
      const float4 a = tile[j];
      const float4 b = tile[j + 1];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const float ta = fmaf(px[r], a.x, fmaf(py[r], a.y, fmaf(pz[r], a.z, a.w)));
        const float tb = fmaf(px[r], b.x, fmaf(py[r], b.y, fmaf(pz[r], b.z, b.w)));
        tt[r] = min3f(tt[r], ta, tb);
      }
    }
    bool hit = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      hit |= ok[r] && pp[r] + tt[r] < thr;
      tmin[r] = fminf(tmin[r], tt[r]);
    }
    if (__syncthreads_or(hit) && tid == 0)
      append_block_hits(S, qb, base / kTilePts, red, pass_b_reach2(thr, S.d_max));
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t slot = (int64_t)qb * kQueriesPerBlock + r * kBlock + tid;
    if (ok[r]) atomicMin(S.out_slot + slot, __float_as_uint(fmaxf(pp[r] + tmin[r], 0.0f)));
  }
}

// Compact the queries of two-pass sets whose pass-A value is under the bound into
// the list segment of their pass-A block.
// Block = 256 consecutive queries of one set; one atomic per block.
__global__ __launch_bounds__(kBlock) void k_flag(const QuerySet* __restrict__ sets, int n_sets) {
  __shared__ int wave_cnt[4];
  __shared__ int base;
  const int64_t bid = blockIdx.x;
  // query_base holds the prefix of ceil(Q / kBlock) blocks over sets
  const int s = find_owner(sets, n_sets, bid, [](const QuerySet& q) { return q.query_base; });
  const QuerySet S = sets[s];  // a copy: the stores below cannot alias it
  // pass-A slots in order; the query of a slot comes from the spatial sort
  const int64_t slot = (bid - S.query_base) * kBlock + threadIdx.x;
  bool flag = false;
  if (slot < S.Q) {
    const float d2 = __uint_as_float(S.out_slot[slot]);
    flag = d2 < S.thresh[slot / S.qpbA];
  }
  const uint64_t mask = __ballot(flag);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int before = __popcll(mask & ((1ull << lane) - 1ull));
  if (lane == 0) wave_cnt[w] = __popcll(mask);
  __syncthreads();
  // the block's 256 queries lie in one pass-A block (qpbA is a multiple of 256)
  const int64_t qb = ((bid - S.query_base) * kBlock) / S.qpbA;
  if (threadIdx.x == 0) {
    const int tot = wave_cnt[0] + wave_cnt[1] + wave_cnt[2] + wave_cnt[3];
    base = tot ? atomicAdd(S.seg_count + qb, tot) : 0;
  }
  __syncthreads();
  if (flag) {
    int off = base + before;
    for (int i = 0; i < w; ++i) off += wave_cnt[i];
    const int64_t e = qb * S.qpbA + off;
    S.list[e] = (int32_t)slot;
    S.fpos[e] = make_float4(S.sp[slot], S.sp[S.Q + slot], S.sp[2 * S.Q + slot],
                            0.0f);  // read back by pass B
    S.out_slot[slot] = kInfBits;
    if (S.nn) S.nn[e] = ~0ull;
  }
}

// Nearest indices of the flagged queries (sets with nn), persistent grid over the
// segment slots of every query block.
__global__ __launch_bounds__(kBlock) void k_scatter_nearest(const QuerySet* __restrict__ sets,
                                                            int n_sets) {
  for (int s = 0; s < n_sets; ++s) {
    const QuerySet S = sets[s];  // a copy: the stores below cannot alias it
    if (!S.nn || !S.list) continue;
    const int64_t slots = (int64_t)S.n_qblocks * S.qpbA;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < slots;
         i += (int64_t)gridDim.x * kBlock) {
      const int64_t qb = i / S.qpbA;
      if (i - qb * S.qpbA >= S.seg_count[qb]) continue;
      const unsigned long long v = S.nn[i];
      const unsigned idx = (unsigned)(v & 0xffffffffull);
      S.nidx[perm_query(S, S.list[i])] =
          (v == ~0ull || idx >= (unsigned)S.n_points) ? -1 : (int32_t)idx;
    }
  }
}

}  // namespace

hipError_t launch_min_dist(const QuerySet* d_sets, int n_sets, int64_t total_blocks,
                           hipStream_t s) {
  if (total_blocks > 0) k_min_dist_exact<<<(unsigned)total_blocks, kBlock, 0, s>>>(d_sets, n_sets);
  return hipGetLastError();
}

hipError_t launch_min_dist_approx(const QuerySet* d_sets, int n_sets, int64_t total_blocks,
                                  int variant, hipStream_t s) {
  if (total_blocks > 0) {
    if (variant == kPassAMfma || variant == kPassAF16s)
      return launch_min_dist_approx_matrix(d_sets, n_sets, total_blocks, variant, s);
    k_min_dist_approx<<<(unsigned)total_blocks, kBlock, 0, s>>>(d_sets, n_sets);
  }
  return hipGetLastError();
}

hipError_t launch_flag(const QuerySet* d_sets, int n_sets, int64_t total_blocks, hipStream_t s) {
  if (total_blocks > 0) k_flag<<<(unsigned)total_blocks, kBlock, 0, s>>>(d_sets, n_sets);
  return hipGetLastError();
}

hipError_t launch_scatter_nearest(const QuerySet* d_sets, int n_sets, hipStream_t s) {
  k_scatter_nearest<<<256, kBlock, 0, s>>>(d_sets, n_sets);
  return hipGetLastError();
}

hipError_t launch_min_dist_listed(const QuerySet* d_sets, int n_sets, int64_t max_items,
                                  hipStream_t s) {
  if (max_items > 0) {
    const int64_t sub = max_items * kTileSplit;  // entries expand into their sub-tiles
    const unsigned grid = (unsigned)(sub < kPersistBlocks ? sub : kPersistBlocks);
    k_min_dist_listed<<<grid, kBlock, 0, s>>>(d_sets, n_sets);
  }
  return hipGetLastError();
}

}  // namespace aero
