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
// positions as the flag kernel wrote them) against the points of one cloud sub-tile
// (raw or sorted order).  With kIdx also the lowest point index attaining the
// minimum (the sorted order visits indices in any order, so ties compare indices).
template <int R, bool kIdx>
__device__ inline void listed_item(const QuerySet& S, int64_t qb, int cnt, unsigned ys,
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
  float x, y, z;
  int32_t idx;
  bool in;
  int n;
  item_point(S, ys, x, y, z, idx, in, n);
  // every thread writes its own slot (a far record past the sub-tile's points), so an
  // odd count still leaves a valid record after the last point
  tile[tid] = in ? make_float4(x, y, z, __int_as_float(idx))
                 : make_float4(kFar, kFar, kFar, __int_as_float(0x7fffffff));
  const int n2 = (n + 1) & ~1;  // even: the loop takes points in pairs
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
        const int32_t ia = __float_as_int(a.w), ic = __float_as_int(c.w);
        if (da < best[r] || (da == best[r] && ia < bidx[r])) {
          best[r] = da;
          bidx[r] = ia;
        }
        if (dc < best[r] || (dc == best[r] && ic < bidx[r])) {
          best[r] = dc;
          bidx[r] = ic;
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
__device__ inline void listed_item_r(const QuerySet& S, int64_t qb, int cnt, unsigned ys,
                                     float4* tile) {
  if (S.nn)
    listed_item<R, true>(S, qb, cnt, ys, tile);
  else
    listed_item<R, false>(S, qb, cnt, ys, tile);
}

// Pass B: exact direct form for the flagged queries, only against the items (block,
// sub-tile) that pass A marked for their block (a query's nearest point within d_max
// always lies in one).  Persistent grid over the call's item list, whose length is
// read on the device.
__global__ __launch_bounds__(kBlock) void k_min_dist_listed(const QuerySet* __restrict__ sets,
                                                            int n_sets,
                                                            const int2* __restrict__ items,
                                                            const int32_t* __restrict__ item_count,
                                                            const unsigned char* __restrict__ hitf) {
  __shared__ float4 tile[kSubPts];
  const int64_t total = *item_count;
  SetCache cache{0, 0, 0};
  for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
    if (!hitf[it]) continue;  // block-uniform
    const int2 e = items[it];
    const int s = set_of(sets, n_sets, e.x, cache);
    const QuerySet S = sets[s];
    if (!block_of(S, e.x) || !S.list) continue;
    const int64_t qb = e.x - S.qb_base;
    const int cnt = min(S.seg_count[qb], S.qpbA);
    if (cnt <= 0) continue;
    const int nr = (cnt + kBlock - 1) / kBlock;
    // exactly as many flagged queries per lane as the block has (no idle groups)
    switch (nr) {
      case 1: listed_item_r<1>(S, qb, cnt, (unsigned)e.y, tile); break;
      case 2: listed_item_r<2>(S, qb, cnt, (unsigned)e.y, tile); break;
      case 3: listed_item_r<3>(S, qb, cnt, (unsigned)e.y, tile); break;
      case 4: listed_item_r<4>(S, qb, cnt, (unsigned)e.y, tile); break;
      case 5: listed_item_r<5>(S, qb, cnt, (unsigned)e.y, tile); break;
      case 6: listed_item_r<6>(S, qb, cnt, (unsigned)e.y, tile); break;
      case 7: listed_item_r<7>(S, qb, cnt, (unsigned)e.y, tile); break;
      default: listed_item_r<kQueriesPerLane>(S, qb, cnt, (unsigned)e.y, tile); break;
    }
  }
}

// Pass A on the VALU.  Persistent grid over the cull step's item list (see the
// matrix-core pass): a block's kQueriesPerBlock positions are recentred on its
// centre and held in registers (kQueriesPerLane per lane) while the run of its items
// goes by; each item's sub-tile is staged in LDS as (-2 o', |o'|^2) records (double
// buffered), and t = |o'|^2 - 2 p'.o' takes three FMAs and half a min3 per pair.
constexpr int kPassAGridValu = 1024;

__global__ __launch_bounds__(kBlock) void k_pass_a_valu(const QuerySet* __restrict__ sets,
                                                        int n_sets, const int2* __restrict__ items,
                                                        const int32_t* __restrict__ item_count,
                                                        unsigned char* __restrict__ hitf) {
  constexpr int R = kQueriesPerLane;
  __shared__ float4 tile[2][kSubPts];
  const int tid = threadIdx.x;
  const int64_t total = *item_count;
  const int64_t G = gridDim.x;
  const int64_t per = (total + G - 1) / G;
  const int64_t i0 = (int64_t)blockIdx.x * per, i1 = min<int64_t>(total, i0 + per);
  if (i0 >= i1) return;  // block-uniform
  SetCache cache{0, 0, 0};
  int64_t cur = -1, slot0 = 0;
  unsigned* out_slot = nullptr;
  unsigned okm = 0;  // bit r: this lane's query r exists
  float c[3] = {0.0f, 0.0f, 0.0f}, thr = 0.0f;
  float px[R], py[R], pz[R], pp[R], tmin[R];
  auto flush = [&]() {
#pragma unroll
    for (int r = 0; r < R; ++r)
      if ((okm >> r) & 1u)
        atomicMin(out_slot + slot0 + r * kBlock, __float_as_uint(fmaxf(pp[r] + tmin[r], 0.0f)));
  };
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
    if (ivalid && gqb != cur) {  // block-uniform
      if (cur >= 0) flush();
      const QuerySet& S = sets[ns];
      const int64_t qb = gqb - S.qb_base;
      const int64_t Q = S.Q;
      const float* __restrict__ sp = S.sp;
      out_slot = S.out_slot;
      const float4 bi = S.binfo[qb];
      c[0] = bi.x;
      c[1] = bi.y;
      c[2] = bi.z;
      thr = bi.w;
      slot0 = qb * kQueriesPerBlock + tid;
      okm = 0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int64_t slot = slot0 + r * kBlock;
        const bool ok = slot < Q;
        okm |= ok ? 1u << r : 0u;
        const int64_t qs = ok ? slot : 0;  // positions in slot order
        px[r] = sp[qs] - c[0];
        py[r] = sp[Q + qs] - c[1];
        pz[r] = sp[2 * Q + qs] - c[2];
        pp[r] = fmaf(pz[r], pz[r], fmaf(py[r], py[r], px[r] * px[r]));
        tmin[r] = kFarT;
      }
      cur = gqb;
    }
    if (ivalid) {
      const float x = ox - c[0], y = oy - c[1], z = oz - c[2];
      tile[buf][tid] = oin ? make_float4(-2.0f * x, -2.0f * y, -2.0f * z,
                                         fmaf(z, z, fmaf(y, y, x * x)))
                           : make_float4(0.0f, 0.0f, 0.0f, kFarT);
    }
    if (i + 1 < i1) {
      it = items[i + 1];
      ns = set_of(sets, n_sets, it.x, cache);
      item_point(sets[ns], (unsigned)it.y, ox, oy, oz, oidx, oin, cnt);
      valid = block_of(sets[ns], it.x) && cnt > 0;
    }
    if (!ivalid) continue;  // block-uniform; the buffers alternate over processed items only
    __syncthreads();
    const float4* tl = tile[buf];
    buf ^= 1;
    float tt[R];
#pragma unroll
    for (int r = 0; r < R; ++r) tt[r] = kFarT;
    const int cnt2 = (icnt + 1) & ~1;  // pairs; an odd tail reads a far record
#pragma unroll 4
    for (int j = 0; j < cnt2; j += 2) {
      const float4 a = tl[j];
      const float4 b = tl[j + 1];
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
      hit |= ((okm >> r) & 1u) && pp[r] + tt[r] < thr;
      tmin[r] = fminf(tmin[r], tt[r]);
    }
    mark_hit(hit, hitf, i);
  }
  if (cur >= 0) flush();
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

hipError_t launch_pass_a(const QuerySet* d_sets, int n_sets, const int2* items,
                         const int32_t* item_count, unsigned char* hitf, int64_t max_items,
                         int variant, hipStream_t s) {
  if (max_items <= 0) return hipSuccess;
  if (variant == kPassAF16s4 || variant == kPassAF16s8)
    return launch_pass_a_matrix(d_sets, n_sets, items, item_count, hitf, max_items, variant, s);
  const unsigned grid = (unsigned)(max_items < kPassAGridValu ? max_items : kPassAGridValu);
  k_pass_a_valu<<<grid, kBlock, 0, s>>>(d_sets, n_sets, items, item_count, hitf);
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

hipError_t launch_min_dist_listed(const QuerySet* d_sets, int n_sets, const int2* items,
                                  const int32_t* item_count, const unsigned char* hitf,
                                  int64_t max_items, hipStream_t s) {
  if (max_items > 0) {
    const unsigned grid = (unsigned)(max_items < kPersistBlocks ? max_items : kPersistBlocks);
    k_min_dist_listed<<<grid, kBlock, 0, s>>>(d_sets, n_sets, items, item_count, hitf);
  }
  return hipGetLastError();
}

}  // namespace aero
