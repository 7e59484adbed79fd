// Nearest squared distance from rollout positions to the raw cloud (the d_t of the
// collision cost, Sec. IV-C).
//
//   k_min_dist_exact   direct form (p - o)^2 per pair over every query of a set and
//                      the cloud tiles within d_max of its wave's queries (Stage II);
//                      cloud tiles staged in LDS with their boxes and read as wave-
//                      wide broadcasts, queries in registers.
//   k_pass_a_valu      pass A over the cull step's (query block, sub-tile) items: the
//                      expanded form |o'|^2 - 2 p'.o' with query and cloud recentred on
//                      the block's centre, three FMAs and half a min3 per pair; per
//                      item, the hit words of the queries that came under the block's
//                      bound, and each query's least value over its hit items (the
//                      matrix-core variants live in distance_mfma.hip).
//   k_pass_b           pass B: the direct form for the (query, sub-tile) pairs of the
//                      hit words, skipping the sub-tile's 32-point groups that lie
//                      beyond every listed query's cap (its least pass-A value plus
//                      the block's error allowance, or d_max).
//   k_scatter_nearest  nearest indices from pass B's records (when requested).
//
// Results combine through atomicMin on the float bit patterns of the non-negative
// squared distances (exact and order independent), so every result is bitwise
// reproducible.  A query that no pass-B pair reaches keeps +inf: its pass-A values
// stayed over the bound everywhere, so its distance is provably >= d_max, where the
// collision penalty is 0 whatever the exact value.
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

// Direct-form min over the cloud points [g0, g1) for R queries per lane, the wave's
// queries lying in the box [qlo, qhi].  Each tile of kTilePts points is staged in LDS
// with its bounding box; a wave skips a tile whose box lies farther than d_max from
// its queries' box (squared limit `lim`, rounding margin included): no pair of that
// tile can come under d_max, and from d_max on the collision penalty is 0, so such a
// query's result only has to stay >= d_max^2 (+inf when no tile was evaluated).
template <int R>
__device__ inline void direct_range(const QuerySet& S, int64_t g0, int64_t g1, float4* tile,
                                    float* tbox, const float qlo[3], const float qhi[3],
                                    float lim, const float* px, const float* py,
                                    const float* pz, float* best) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  constexpr int kStep = 8;  // points per step of the pair loop (LDS reads issued together)
  static_assert(kTilePts % kStep == 0, "a tile holds whole steps");
  for (int64_t base = g0; base < g1; base += kTilePts) {
    const int cnt = (int)min<int64_t>(kTilePts, g1 - base);
    const int cnt8 = (cnt + kStep - 1) / kStep * kStep;  // padded with far points
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int pt = tid; pt < cnt8; pt += kBlock) {
      const int64_t g = base + pt;
      const bool in = pt < cnt;
      const int64_t gg = in ? g : base;  // always a valid address
      const float x = S.cloud[3 * gg], y = S.cloud[3 * gg + 1], z = S.cloud[3 * gg + 2];
      tile[pt] = in ? make_float4(x, y, z, 0.0f) : make_float4(kFar, kFar, kFar, 0.0f);
      lo[0] = fminf(lo[0], x);
      lo[1] = fminf(lo[1], y);
      lo[2] = fminf(lo[2], z);
      hi[0] = fmaxf(hi[0], x);
      hi[1] = fmaxf(hi[1], y);
      hi[2] = fmaxf(hi[2], z);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = wave_minf(lo[a]);
      hi[a] = wave_maxf(hi[a]);
    }
    if (lane == 0)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        tbox[6 * w + a] = lo[a];
        tbox[6 * w + 3 + a] = hi[a];
      }
    __syncthreads();
    float b[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      b[a] = tbox[a];
      b[3 + a] = tbox[3 + a];
#pragma unroll
      for (int v = 1; v < kBlock / 64; ++v) {
        b[a] = fminf(b[a], tbox[6 * v + a]);
        b[3 + a] = fmaxf(b[3 + a], tbox[6 * v + 3 + a]);
      }
    }
    if (box_dist2(b, qlo, qhi) <= lim) {  // the same for every lane of the wave
      for (int j = 0; j < cnt8; j += kStep) {
        float4 o[kStep];
#pragma unroll
        for (int i = 0; i < kStep; ++i) o[i] = tile[j + i];
#pragma unroll
        for (int i = 0; i < kStep; i += 2)
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const float ax = px[r] - o[i].x, ay = py[r] - o[i].y, az = pz[r] - o[i].z;
            const float cx = px[r] - o[i + 1].x, cy = py[r] - o[i + 1].y, cz = pz[r] - o[i + 1].z;
            const float da = fmaf(az, az, fmaf(ay, ay, ax * ax));
            const float dc = fmaf(cz, cz, fmaf(cy, cy, cx * cx));
            best[r] = min3f(best[r], da, dc);
          }
      }
    }
    __syncthreads();
  }
}

// Every query of an exact set.  Block = (query block of R * kBlock queries, cloud
// chunk); R (queries per lane) is sized to the set, so that small sets leave few
// lanes idle.  Wave w takes the block's queries [w R 64, (w + 1) R 64), consecutive
// positions of a few rollouts, so that their box is small.
template <int R>
__device__ inline void exact_block(const QuerySet& S, int qb, int ch, float lim, float4* tile,
                                   float* tbox) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t q0 = (int64_t)qb * (R * kBlock) + (int64_t)w * (R * 64) + lane;
  float px[R], py[R], pz[R], best[R];
  float qlo[3] = {INFINITY, INFINITY, INFINITY}, qhi[3] = {-INFINITY, -INFINITY, -INFINITY};
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t q = q0 + r * 64;
    const int64_t qq = q < S.Q ? q : 0;  // out-of-range lanes read query 0, never stored
    px[r] = S.px[qq];
    py[r] = S.py[qq];
    pz[r] = S.pz[qq];
    best[r] = __uint_as_float(kInfBits);
    if (q < S.Q) {
      qlo[0] = fminf(qlo[0], px[r]);
      qlo[1] = fminf(qlo[1], py[r]);
      qlo[2] = fminf(qlo[2], pz[r]);
      qhi[0] = fmaxf(qhi[0], px[r]);
      qhi[1] = fmaxf(qhi[1], py[r]);
      qhi[2] = fmaxf(qhi[2], pz[r]);
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    qlo[a] = wave_minf(qlo[a]);
    qhi[a] = wave_maxf(qhi[a]);
  }
  const int64_t g0 = (int64_t)ch * S.chunk_pts;
  const int64_t g1 = min<int64_t>(g0 + S.chunk_pts, S.n_points);
  direct_range<R>(S, g0, g1, tile, tbox, qlo, qhi, lim, px, py, pz, best);
  unsigned* out = S.out + (int64_t)(blockIdx.x % max(S.n_copies, 1)) * S.Q;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t q = q0 + r * 64;
    // the outputs start at +inf: a query no evaluated pair reached has nothing to add
    if (q < S.Q && best[r] < __uint_as_float(kInfBits)) atomicMin(out + q, __float_as_uint(best[r]));
  }
}

__global__ __launch_bounds__(kBlock) void k_min_dist_exact(const QuerySet* __restrict__ sets,
                                                           int n_sets, float lim) {
  __shared__ float4 tile[kTilePts];
  __shared__ float tbox[6 * (kBlock / 64)];
  const int64_t bid = blockIdx.x;
  const int s = find_owner(sets, n_sets, bid, [](const QuerySet& q) { return q.block_base; });
  const QuerySet S = sets[s];
  const int64_t local = bid - S.block_base;
  const int qb = (int)(local / S.n_chunks), ch = (int)(local % S.n_chunks);
  switch (S.qpbA / kBlock) {  // block-uniform
    case 1: exact_block<1>(S, qb, ch, lim, tile, tbox); break;
    case 2: exact_block<2>(S, qb, ch, lim, tile, tbox); break;
    case 4: exact_block<4>(S, qb, ch, lim, tile, tbox); break;
    default: exact_block<kQueriesPerLane>(S, qb, ch, lim, tile, tbox); break;
  }
}


// Pass B: the exact direct form (p - o)^2 for the (query, sub-tile) pairs that pass A
// marked: for a marked item, the queries of its block whose pass-A value came under
// the bound in its sub-tile (all of the block's queries for an item without room
// for its hit words).  A query's nearest point within d_max lies in such a sub-tile
// (its pass-A value there is under the bound), and every other point of the reach is
// farther than d_max, so the minimum over the evaluated pairs is exact below d_max.
//
// Each wave works alone (no workgroup barriers): waves take the marked items in turn
// (items strided over every wave of the grid), list the item's hit queries from its
// words into the wave's own LDS row and, per listed query, the sub-tile's 32-point
// groups within the query's cap (see pass_b_cap).  Group by group, the wave then runs
// the queries that need the group, up to kPassBRows of them per lane, against the
// group's points, which every lane reads at the same address: through the constant
// address space (the points are not written while the kernel runs), so they arrive
// as scalar loads into SGPRs and cost no LDS bandwidth and no vector-memory issue.
// Results combine through minima on float bits (and on (d^2 bits, index) pairs for
// the nearest index, lowest index on ties), in LDS per unit and then by atomicMin in
// device memory, so they are order independent.
#ifndef AERO_PASS_B_ROWS
#define AERO_PASS_B_ROWS AERO_QUERIES_PER_LANE
#endif
constexpr int kPassBRows = AERO_PASS_B_ROWS;  // listed queries per lane at a time

typedef const __attribute__((address_space(4))) float cfloat;
typedef const __attribute__((address_space(4))) int32_t cint;

// One point (x, y, z, index) against the R queries of this lane.
template <int R, bool kIdx>
__device__ __forceinline__ void pass_b_point(float ox, float oy, float oz, int32_t oi,
                                             const float* px, const float* py, const float* pz,
                                             float* best, int32_t* bidx) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const float ax = px[r] - ox, ay = py[r] - oy, az = pz[r] - oz;
    const float d = fmaf(az, az, fmaf(ay, ay, ax * ax));
    if constexpr (kIdx) {  // branch-free: no short-circuit evaluation
      const bool take = (d < best[r]) | ((d == best[r]) & (oi < bidx[r]));
      bidx[r] = take ? oi : bidx[r];
      best[r] = take ? d : best[r];
    } else {
      best[r] = fminf(best[r], d);
    }
  }
}

// The group-skipping bound of pass B: a group box at single-precision squared distance
// of at least this from a query holds only points whose single-precision squared
// distance exceeds d_max^2.  The box distance and a point's direct-form distance
// each carry a relative error of at most about 5 units in the last place (exact
// differences of floats rounded once, then one multiply and two fused adds), and
// every point lies at least as far as the box, so a margin of 2^-19 relative
// (32 units) suffices; the result is rounded up to single precision.
__device__ inline float pass_b_reach(float d_max) {
  const double r = (double)d_max * (double)d_max * (1.0 + 0x1p-19);
  const float f = (float)r;
  return (double)f >= r ? f : __uint_as_float(__float_as_uint(f) + 1u);
}

// The cap of pass B on a query's squared distances: a point group whose box lies at
// least this far holds no point that can be the query's nearest.  m is the query's
// least pass-A value (clamped at 0) over its hit items and slack the block's
// allowance for pass A's error (its bound less d_max^2): the point attaining m lies
// within m + slack exactly, so its direct-form value does too up to the relative
// margin above, and every point of a farther group exceeds it.
__device__ inline float pass_b_cap(float m, float slack) {
  return (m + slack) * (1.0f + 0x1p-19f);
}

// A wave's LDS record of a listed query's least value: the float bits of d^2, or
// (d^2 bits << 32 | point index) when nearest indices are kept; all ones: none yet.
template <bool kIdx>
struct PassBBest {
  typedef unsigned T;
};
template <>
struct PassBBest<true> {
  typedef unsigned long long T;
};

constexpr int kUnitQ = 64 * kQueriesPerLane;  // the most listed queries of a work unit
static_assert(kGroupsPerSub <= 8, "a row's group mask holds 8 bits");

// Queries of one point group: entries c0 + r * 64 + lane (r < R, below ng) of the
// group's list, each an index into the unit's list of block-local queries, against
// the group's n points from point g0 on (sorted records, or the raw cloud).  Every
// lane reads the same point at a time, through the constant address space (scalar
// loads into SGPRs).  Each query's least value joins its LDS record (an entry occurs
// once in a group's list, so the records' minima do not race).
template <int R, bool kIdx, bool kSorted>
__device__ inline void pass_b_group(const QuerySet& S, int64_t slot0, const uint16_t* qlist,
                                    const uint16_t* glist, int c0, int ng, int64_t g0, int n,
                                    typename PassBBest<kIdx>::T* bl) {
  constexpr int U = R <= 2 ? 4 : 2;
  const int lane = threadIdx.x & 63;
  const int64_t Q = S.Q;
  const float* __restrict__ sp = S.sp;
  float px[R], py[R], pz[R], best[R];
  int32_t bidx[R], e[R];  // e: the unit-list entry, -1 for an idle row
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int k = c0 + r * 64 + lane;
    e[r] = k < ng ? (int32_t)glist[k] : -1;
    const int64_t q = slot0 + (e[r] >= 0 ? qlist[e[r]] : 0);  // always a valid position
    px[r] = sp[q];
    py[r] = sp[Q + q];
    pz[r] = sp[2 * Q + q];
    best[r] = __uint_as_float(kInfBits);
    bidx[r] = 0x7fffffff;
  }
  if constexpr (kSorted) {
    cfloat* rec = (cfloat*)(S.scloud + g0);  // (x, y, z, index bits) per point
    cint* irec = (cint*)(S.scloud + g0);
    int j = 0;
    for (; j + U <= n; j += U) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        pass_b_point<R, kIdx>(rec[4 * (j + u)], rec[4 * (j + u) + 1], rec[4 * (j + u) + 2],
                              irec[4 * (j + u) + 3], px, py, pz, best, bidx);
    }
    for (; j < n; ++j)
      pass_b_point<R, kIdx>(rec[4 * j], rec[4 * j + 1], rec[4 * j + 2], irec[4 * j + 3], px, py,
                            pz, best, bidx);
  } else {
    cfloat* rec = (cfloat*)(S.cloud + 3 * g0);
    int j = 0;
    for (; j + U <= n; j += U) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        pass_b_point<R, kIdx>(rec[3 * (j + u)], rec[3 * (j + u) + 1], rec[3 * (j + u) + 2],
                              (int32_t)(g0 + j + u), px, py, pz, best, bidx);
    }
    for (; j < n; ++j)
      pass_b_point<R, kIdx>(rec[3 * j], rec[3 * j + 1], rec[3 * j + 2], (int32_t)(g0 + j), px,
                            py, pz, best, bidx);
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (e[r] < 0) continue;
    if constexpr (kIdx)
      atomicMin(bl + e[r], ((unsigned long long)__float_as_uint(best[r]) << 32) |
                               (unsigned long long)(unsigned)bidx[r]);
    else
      atomicMin(bl + e[r], __float_as_uint(best[r]));
  }
}

// Orders this wave's LDS accesses (lists and records are written and read by the
// wave alone, across lanes).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The groups of the sub-tile (n points; gb: its group boxes, or nullptr for every
// group) within the cap of the query at slot q: bit g for group g.
__device__ inline uint32_t pass_b_group_mask(const QuerySet& S, int64_t q, const float* gb,
                                             int n, float reach, float slack) {
  if (!gb) return (1u << ((n + 31) / 32)) - 1u;
  const int64_t Q = S.Q;
  const float x = S.sp[q], y = S.sp[Q + q], z = S.sp[2 * Q + q];
  const float lim =
      S.amin ? fminf(reach, pass_b_cap(__uint_as_float(S.amin[q]), slack)) : reach;
  cfloat* gbc = (cfloat*)gb;
  uint32_t m = 0;
#pragma unroll
  for (int g = 0; g < kGroupsPerSub; ++g) {
    cfloat* bx = gbc + 6 * g;
    const float dx = fmaxf(fmaxf(bx[0] - x, x - bx[3]), 0.0f);
    const float dy = fmaxf(fmaxf(bx[1] - y, y - bx[4]), 0.0f);
    const float dz = fmaxf(fmaxf(bx[2] - z, z - bx[5]), 0.0f);
    m |= fmaf(dz, dz, fmaf(dy, dy, dx * dx)) < lim ? 1u << g : 0u;
  }
  return m;
}

// A unit of a single row (hu <= 64 listed queries, one per lane): the row's queries
// stay in registers across the groups, and a group runs when some query of the row
// needs it (with one row there is nothing to compact).  One device-memory minimum per
// query at the end.
template <bool kIdx, bool kSorted>
__device__ inline void pass_b_row(const QuerySet& S, int64_t slot0, const uint16_t* qlist,
                                  int hu, int64_t g0, int n, const float* gb, float reach,
                                  float slack) {
  const int lane = threadIdx.x & 63;
  const int64_t Q = S.Q;
  const bool on = lane < hu;
  const int64_t q = slot0 + (on ? qlist[lane] : qlist[0]);  // always a valid position
  float px[1] = {S.sp[q]}, py[1] = {S.sp[Q + q]}, pz[1] = {S.sp[2 * Q + q]};
  float best[1] = {__uint_as_float(kInfBits)};
  int32_t bidx[1] = {0x7fffffff};
  const uint32_t m = on ? pass_b_group_mask(S, q, gb, n, reach, slack) : 0u;
  const int ngr = (n + 31) / 32;
  for (int g = 0; g < ngr; ++g) {  // wave-uniform
    if (!__builtin_amdgcn_ballot_w64((m >> g) & 1u)) continue;
    const int64_t gg = g0 + 32 * g;
    const int gn = min(32, n - 32 * g);
    if constexpr (kSorted) {
      cfloat* rec = (cfloat*)(S.scloud + gg);
      cint* irec = (cint*)(S.scloud + gg);
      int j = 0;
      for (; j + 4 <= gn; j += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
          pass_b_point<1, kIdx>(rec[4 * (j + u)], rec[4 * (j + u) + 1], rec[4 * (j + u) + 2],
                                irec[4 * (j + u) + 3], px, py, pz, best, bidx);
      }
      for (; j < gn; ++j)
        pass_b_point<1, kIdx>(rec[4 * j], rec[4 * j + 1], rec[4 * j + 2], irec[4 * j + 3], px,
                              py, pz, best, bidx);
    } else {
      cfloat* rec = (cfloat*)(S.cloud + 3 * gg);
      int j = 0;
      for (; j + 4 <= gn; j += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
          pass_b_point<1, kIdx>(rec[3 * (j + u)], rec[3 * (j + u) + 1], rec[3 * (j + u) + 2],
                                (int32_t)(gg + j + u), px, py, pz, best, bidx);
      }
      for (; j < gn; ++j)
        pass_b_point<1, kIdx>(rec[3 * j], rec[3 * j + 1], rec[3 * j + 2], (int32_t)(gg + j), px,
                              py, pz, best, bidx);
    }
  }
  if (!on || best[0] == __uint_as_float(kInfBits)) return;  // no group within the cap
  atomicMin(S.out_slot + q, __float_as_uint(best[0]));
  if constexpr (kIdx)
    atomicMin(S.nn + q, ((unsigned long long)__float_as_uint(best[0]) << 32) |
                            (unsigned long long)(unsigned)bidx[0]);
}

// One work unit: the hu listed queries of qlist (block-local indices) against the
// item's sub-tile (n points from point g0 on; gb: its group boxes, or nullptr to take
// every group).  Each query takes only the groups within its cap, so the wave runs
// group by group, each over the compacted list of the queries that need it, and
// every query's least value meets in LDS before one global minimum per query.
template <bool kIdx, bool kSorted>
__device__ inline void pass_b_unit(const QuerySet& S, int64_t slot0, const uint16_t* qlist,
                                   int hu, int64_t g0, int n, const float* gb, float reach,
                                   float slack, uint16_t* glist,
                                   typename PassBBest<kIdx>::T* bl) {
  typedef typename PassBBest<kIdx>::T BestT;
  if (hu <= 64) {  // wave-uniform
    pass_b_row<kIdx, kSorted>(S, slot0, qlist, hu, g0, n, gb, reach, slack);
    return;
  }
  const int lane = threadIdx.x & 63;
  const int nr = (hu + 63) / 64;     // rows of the unit
  const int ngr = (n + 31) / 32;     // groups of the sub-tile
  // group masks, 8 bits per row: bit g of row r, group g within the cap of query
  // r * 64 + lane
  uint64_t gm = 0;
  for (int r = 0; r < nr; ++r) {  // wave-uniform
    const int k = r * 64 + lane;
    if (k >= hu) continue;
    bl[k] = ~BestT(0);
    gm |= (uint64_t)pass_b_group_mask(S, slot0 + qlist[k], gb, n, reach, slack) << (8 * r);
  }
  for (int g = 0; g < ngr; ++g) {  // wave-uniform
    // the list of the queries that need group g
    wave_lds_sync();  // the previous group's readers are done with the list
    int ng = 0;
    for (int r = 0; r < nr; ++r) {
      const bool bit = (gm >> (8 * r + g)) & 1ull;
      const uint64_t bal = __builtin_amdgcn_ballot_w64(bit);
      if (bit) glist[ng + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                 __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u))] =
          (uint16_t)(r * 64 + lane);
      ng += __popcll(bal);
    }
    if (ng == 0) continue;
    wave_lds_sync();
    const int64_t gg = g0 + 32 * g;
    const int gn = min(32, n - 32 * g);
    for (int c0 = 0; c0 < ng; c0 += 64 * kPassBRows) {  // wave-uniform
      switch (min((ng - c0 + 63) / 64, kPassBRows)) {
        case 1: pass_b_group<1, kIdx, kSorted>(S, slot0, qlist, glist, c0, ng, gg, gn, bl); break;
        case 2: pass_b_group<2, kIdx, kSorted>(S, slot0, qlist, glist, c0, ng, gg, gn, bl); break;
        case 3: pass_b_group<3, kIdx, kSorted>(S, slot0, qlist, glist, c0, ng, gg, gn, bl); break;
        case 4: pass_b_group<4, kIdx, kSorted>(S, slot0, qlist, glist, c0, ng, gg, gn, bl); break;
        case 5: pass_b_group<5, kIdx, kSorted>(S, slot0, qlist, glist, c0, ng, gg, gn, bl); break;
        case 6: pass_b_group<6, kIdx, kSorted>(S, slot0, qlist, glist, c0, ng, gg, gn, bl); break;
        case 7: pass_b_group<7, kIdx, kSorted>(S, slot0, qlist, glist, c0, ng, gg, gn, bl); break;
        default:
          pass_b_group<kPassBRows, kIdx, kSorted>(S, slot0, qlist, glist, c0, ng, gg, gn, bl);
          break;
      }
    }
  }
  wave_lds_sync();  // every group's minima are in
  for (int r = 0; r < nr; ++r) {
    const int k = r * 64 + lane;
    if (k >= hu) continue;
    const BestT v = bl[k];
    if (v == ~BestT(0)) continue;  // no group of this sub-tile within the query's cap
    const int64_t slot = slot0 + qlist[k];
    if constexpr (kIdx) {
      atomicMin(S.out_slot + slot, (unsigned)(v >> 32));
      atomicMin(S.nn + slot, v);
    } else {
      atomicMin(S.out_slot + slot, v);
    }
  }
}

// One work unit of pass B as its pair count takes it (the same steps as k_pass_b,
// which keeps them inline: its registers are at the budget of eight waves per SIMD):
// part `part` of item `it` (e, of set S) covers the item's listed queries
// [part * 64 urows, (part + 1) * 64 urows), listed into qlist (the wave's LDS row).
// Returns false when the unit has nothing to run.
struct PassBUnit {
  int64_t slot0, g0;
  const float* gb;
  int n, hu;
  float reach, slack;
  bool srt;
};
__device__ __forceinline__ bool pass_b_take_unit(const QuerySet& S, int2 e,
                                                 const uint32_t* __restrict__ hmask,
                                                 int64_t mask_words, int64_t it, int part,
                                                 int urows, uint16_t* qlist, PassBUnit& U) {
  const int lane = threadIdx.x & 63;
  if (!block_of(S, e.x) || S.n_points <= 0) return false;
  const int64_t qb = e.x - S.qb_base;
  U.slot0 = qb * S.qpbA;
  const int nq = (int)min<int64_t>(S.qpbA, S.Q - U.slot0);  // queries of the block
  const int W = S.qpbA / 32;
  const unsigned ys = (unsigned)e.y;
  U.g0 = (int64_t)(ys & 0x7fffffffu) * kSubPts;
  U.srt = (ys >> 31) != 0 && S.scloud;
  U.n = U.g0 < S.n_points ? (int)min<int64_t>(kSubPts, S.n_points - U.g0) : 0;
  if (U.n <= 0) return false;
  // the hit queries: lane j holds word j (bits of existing queries only)
  const int lo = lane * 32;
  const uint32_t valid = lo >= nq ? 0u : (nq - lo >= 32 ? 0xffffffffu : (1u << (nq - lo)) - 1u);
  uint32_t word = 0;
  if (lane < W)  // without room for the item's words: every query of the block
    word = (it + 1) * W <= mask_words ? hmask[it * W + lane] & valid : valid;
  const int c = __popc(word);
  int incl = c;  // inclusive scan over the wave
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y2 = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y2;
  }
  const int h = __shfl(incl, 63, 64);
  const int k0 = part * 64 * urows, k1 = min(h, k0 + 64 * urows);
  if (k0 >= k1) return false;  // wave-uniform
  // this unit's part of the list: entries [k0, k1)
  wave_lds_sync();  // the previous unit is done with the row
  int at = incl - c;
  if (at < k1 && incl > k0) {
    while (word) {
      const int b = __ffs(word) - 1;
      word &= word - 1u;
      if (at >= k0 && at < k1) qlist[at - k0] = (uint16_t)(lo + b);
      ++at;
    }
  }
  wave_lds_sync();
  const float* gbs = U.srt ? S.sgbox : S.gbox;
  U.gb = gbs ? gbs + 6 * (int64_t)(ys & 0x7fffffffu) * kGroupsPerSub : nullptr;
  U.reach = pass_b_reach(S.d_max);
  // pass A's error allowance of the block (its bound less d_max^2)
  U.slack = fmaxf(S.binfo[qb].w - S.d_max * S.d_max, 0.0f);
  U.hu = k1 - k0;
  return true;
}

// Work units: whole items (8 rows per unit, the most a lane holds) while the items
// outnumber the waves enough; smaller parts when there are too few items to keep
// every wave busy (the same for every set: one block size per call).
__device__ inline int pass_b_unit_rows(const QuerySet* sets, int64_t total, int64_t n_waves) {
  const int rows_per_block = sets[0].qpbA / 64;
  int urows = kQueriesPerLane;
  while (urows > 1 && total * ((rows_per_block + urows - 1) / urows) < 4 * n_waves) urows /= 2;
  return urows;
}

// kIdx: the call keeps nearest indices (some set has nn; the index-tracking loops need
// more registers, so the plain forward runs its own instantiation).
#ifndef AERO_PASS_B_WPE
#define AERO_PASS_B_WPE 8  // waves per SIMD (at most 64 VGPRs): measured fastest
#endif
template <bool kIdx>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(AERO_PASS_B_WPE))) void
k_pass_b(const QuerySet* __restrict__ sets, int n_sets, const int2* __restrict__ items,
         const int32_t* __restrict__ item_count, const unsigned char* __restrict__ hitf) {
  // each wave's own rows: the unit's listed queries, one group's entries, the records
  __shared__ uint16_t qlists[kBlock / 64][kUnitQ];
  __shared__ uint16_t glists[kBlock / 64][kUnitQ];
  __shared__ typename PassBBest<kIdx>::T bests[kBlock / 64][kUnitQ];
  // the wave index as a wave-uniform value, so that everything derived from it (the
  // item, its set, the point addresses) stays in scalar registers
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint16_t* qlist = qlists[w];
  uint16_t* glist = glists[w];
  const int64_t total = *item_count;
  const int64_t n_waves = (int64_t)gridDim.x * (kBlock / 64);
  const uint32_t* __restrict__ hmask = sets[0].hmask;
  const int64_t mask_words = sets[0].mask_words;
  SetCache cache{0, 0, 0};
  // Work units: part `part` of item it covers the item's listed queries
  // [part * 64 urows, (part + 1) * 64 urows).  Whole items (8 rows per unit, the
  // most a lane holds) while the items outnumber the waves enough; smaller parts
  // when there are too few items to keep every wave busy.
  const int rows_per_block = sets[0].qpbA / 64;  // the same block size for every set
  int urows = kQueriesPerLane;
  while (urows > 1 && total * ((rows_per_block + urows - 1) / urows) < 4 * n_waves) urows /= 2;
  const int parts = (rows_per_block + urows - 1) / urows;
  const int64_t total_units = total * parts;
  for (int64_t u = (int64_t)blockIdx.x * (kBlock / 64) + w; u < total_units; u += n_waves) {
    const int64_t it = u / parts;
    const int part = (int)(u - it * parts);
    if (!hitf[it]) continue;  // wave-uniform
    const int2 e = items[it];
    const int s = set_of(sets, n_sets, e.x, cache);
    const QuerySet S = sets[s];  // a copy: the stores below cannot alias it
    if (!block_of(S, e.x) || S.n_points <= 0) continue;
    const int64_t qb = e.x - S.qb_base;
    const int64_t slot0 = qb * S.qpbA;
    const int nq = (int)min<int64_t>(S.qpbA, S.Q - slot0);  // queries of the block
    const int W = S.qpbA / 32;
    const unsigned ys = (unsigned)e.y;
    const int64_t g0 = (int64_t)(ys & 0x7fffffffu) * kSubPts;
    const bool srt = (ys >> 31) != 0 && S.scloud;
    const int n = g0 < S.n_points ? (int)min<int64_t>(kSubPts, S.n_points - g0) : 0;
    if (n <= 0) continue;
    // the hit queries: lane j holds word j (bits of existing queries only)
    const int lo = lane * 32;
    const uint32_t valid = lo >= nq ? 0u : (nq - lo >= 32 ? 0xffffffffu : (1u << (nq - lo)) - 1u);
    uint32_t word = 0;
    if (lane < W)  // without room for the item's words: every query of the block
      word = (it + 1) * W <= mask_words ? hmask[it * W + lane] & valid : valid;
    const int c = __popc(word);
    int incl = c;  // inclusive scan over the wave
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y2 = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y2;
    }
    const int h = __shfl(incl, 63, 64);
    const int k0 = part * 64 * urows, k1 = min(h, k0 + 64 * urows);
    if (k0 >= k1) continue;  // wave-uniform
    // this unit's part of the list: entries [k0, k1)
    wave_lds_sync();  // the previous unit is done with the rows
    int at = incl - c;
    if (at < k1 && incl > k0) {
      while (word) {
        const int b = __ffs(word) - 1;
        word &= word - 1u;
        if (at >= k0 && at < k1) qlist[at - k0] = (uint16_t)(lo + b);
        ++at;
      }
    }
    wave_lds_sync();
    const float* gbs = srt ? S.sgbox : S.gbox;
    const float* gb = gbs ? gbs + 6 * (int64_t)(ys & 0x7fffffffu) * kGroupsPerSub : nullptr;
    const float reach = pass_b_reach(S.d_max);
    // pass A's error allowance of the block (its bound less d_max^2)
    const float slack = fmaxf(S.binfo[qb].w - S.d_max * S.d_max, 0.0f);
    const int hu = k1 - k0;
    if (kIdx && S.nn) {
      auto* bl = reinterpret_cast<typename PassBBest<kIdx>::T*>(bests[w]);
      if (srt) pass_b_unit<kIdx, true>(S, slot0, qlist, hu, g0, n, gb, reach, slack, glist, bl);
      else pass_b_unit<kIdx, false>(S, slot0, qlist, hu, g0, n, gb, reach, slack, glist, bl);
    } else {
      auto* bl = reinterpret_cast<unsigned*>(bests[w]);
      if (srt) pass_b_unit<false, true>(S, slot0, qlist, hu, g0, n, gb, reach, slack, glist, bl);
      else pass_b_unit<false, false>(S, slot0, qlist, hu, g0, n, gb, reach, slack, glist, bl);
    }
  }
}

// The (query, point) pairs pass B evaluates, for the statistics call: the same work
// units, lists and group masks, summing the points of the groups within each listed
// query's cap into pass_b_pairs.
__device__ unsigned long long pass_b_pairs;
__global__ __launch_bounds__(kBlock) void k_pass_b_count(const QuerySet* __restrict__ sets,
                                                         int n_sets,
                                                         const int2* __restrict__ items,
                                                         const int32_t* __restrict__ item_count,
                                                         const unsigned char* __restrict__ hitf) {
  __shared__ uint16_t qlists[kBlock / 64][kUnitQ];
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint16_t* qlist = qlists[w];
  const int64_t total = *item_count;
  const int64_t n_waves = (int64_t)gridDim.x * (kBlock / 64);
  SetCache cache{0, 0, 0};
  const int urows = pass_b_unit_rows(sets, total, n_waves);
  const int parts = (sets[0].qpbA / 64 + urows - 1) / urows;
  const int64_t total_units = total * parts;
  unsigned long long cnt = 0;
  for (int64_t u = (int64_t)blockIdx.x * (kBlock / 64) + w; u < total_units; u += n_waves) {
    const int64_t it = u / parts;
    if (!hitf[it]) continue;  // wave-uniform
    const int2 e = items[it];
    const QuerySet S = sets[set_of(sets, n_sets, e.x, cache)];
    PassBUnit U;
    if (!pass_b_take_unit(S, e, sets[0].hmask, sets[0].mask_words, it, (int)(u - it * parts),
                          urows, qlist, U))
      continue;
    for (int k = lane; k < U.hu; k += 64) {
      const uint32_t m = pass_b_group_mask(S, U.slot0 + qlist[k], U.gb, U.n, U.reach, U.slack);
      for (int g = 0; g < kGroupsPerSub; ++g)
        if ((m >> g) & 1u) cnt += (unsigned long long)min(32, U.n - 32 * g);
    }
  }
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  if (lane == 0 && cnt) atomicAdd(&pass_b_pairs, cnt);
}

// Pass A on the VALU.  Persistent grid over the cull step's item list (see the
// matrix-core pass): a block's kQueriesPerBlock positions are recentred on its
// centre and held in registers (kQueriesPerLane per lane) while the run of its items
// goes by; each item's sub-tile is staged in LDS as (-2 o', |o'|^2) records (double
// buffered), and t = |o'|^2 - 2 p'.o' takes three FMAs and half a min3 per pair.  Per
// item, the block's queries whose value came under the bound form the item's hit
// words (query r kBlock + tid is bit (r kBlock + tid) % 32 of word
// (r kBlock + tid) / 32).

__global__ __launch_bounds__(kBlock) void k_pass_a_valu(const QuerySet* __restrict__ sets,
                                                        int n_sets, const int2* __restrict__ items,
                                                        const int32_t* __restrict__ item_count,
                                                        unsigned char* __restrict__ hitf) {
  constexpr int R = kQueriesPerLane;
  constexpr int W = kQueriesPerBlock / 32;  // hit words per item
  __shared__ float4 tile[2][kSubPts];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t total = *item_count;
  const int64_t G = gridDim.x;
  const int64_t per = (total + G - 1) / G;
  const int64_t i0 = (int64_t)blockIdx.x * per, i1 = min<int64_t>(total, i0 + per);
  if (i0 >= i1) return;  // block-uniform
  SetCache cache{0, 0, 0};
  int64_t cur = -1;
  unsigned okm = 0;  // bit r: this lane's query r exists
  float c[3] = {0.0f, 0.0f, 0.0f}, thr = 0.0f;
  float px[R], py[R], pz[R], pp[R];
  int64_t qslot0 = 0;        // this lane's slot of row 0
  unsigned* amin = nullptr;  // the block's set's least pass-A values
  // each query's least value over the block's items taken so far by this workgroup
  // (they come in runs): one atomic minimum per query and run instead of per item
  float tmin[R];
#pragma unroll
  for (int r = 0; r < R; ++r) tmin[r] = INFINITY;
  auto flush = [&]() {
    if (amin) {
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (((okm >> r) & 1u) && tmin[r] < thr)  // existing queries that came under
          atomicMin(amin + qslot0 + r * kBlock, __float_as_uint(fmaxf(tmin[r], 0.0f)));
    }
#pragma unroll
    for (int r = 0; r < R; ++r) tmin[r] = INFINITY;
  };
  // the hit words of every set of the call share one array
  AERO_GLOBAL uint32_t* __restrict__ hmask = global_ptr(sets[0].hmask);
  const int64_t mask_items = sets[0].mask_words / W;  // items with room for their words
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
      const int64_t slot0 = qb * kQueriesPerBlock + tid;
      qslot0 = slot0;
      amin = S.amin;
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
    const bool room = i < mask_items;  // block-uniform
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float t = pp[r] + tt[r];
      const bool hq = ((okm >> r) & 1u) && t < thr;
      hit |= hq;
      const uint64_t hb = __ballot(hq);
      if (room && lane < 2)  // the wave's 64 queries r kBlock + 64 w + [0, 64): two words
        hmask[i * W + r * (kBlock / 32) + 2 * w + lane] =
            (uint32_t)(lane ? (hb >> 32) : (hb & 0xffffffffull));
      tmin[r] = fminf(tmin[r], t);
    }
    mark_hit(hit, hitf, i);
  }
  flush();
}

// Nearest indices (sets with nn) from pass B's (d^2 bits, index) records by slot.
__global__ __launch_bounds__(kBlock) void k_scatter_nearest(const QuerySet* __restrict__ sets,
                                                            int n_sets) {
  for (int s = 0; s < n_sets; ++s) {
    const QuerySet S = sets[s];  // a copy: the stores below cannot alias it
    if (!S.nn || !S.items) continue;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < S.Q;
         i += (int64_t)gridDim.x * kBlock) {
      const unsigned long long v = S.nn[i];
      const unsigned idx = (unsigned)(v & 0xffffffffull);
      S.nidx[perm_query(S, i)] = (v == ~0ull || idx >= (unsigned)S.n_points) ? -1 : (int32_t)idx;
    }
  }
}

}  // namespace

hipError_t launch_min_dist(const QuerySet* d_sets, int n_sets, int64_t total_blocks,
                           float d_max, hipStream_t s) {
  // tiles farther than d_max from a wave's queries are skipped; the limit carries a
  // relative margin for the rounding of the box and pair distances
  const float lim = d_max * d_max * (1.0f + 1e-5f) + 1e-6f;
  if (total_blocks > 0)
    k_min_dist_exact<<<(unsigned)total_blocks, kBlock, 0, s>>>(d_sets, n_sets, lim);
  return hipGetLastError();
}

hipError_t launch_pass_a(const QuerySet* d_sets, int n_sets, const int2* items,
                         const int32_t* item_count, unsigned char* hitf, int64_t max_items,
                         int variant, int grid, hipStream_t s) {
  if (max_items <= 0) return hipSuccess;
  if (variant == kPassAF16s4 || variant == kPassAF16s8)
    return launch_pass_a_matrix(d_sets, n_sets, items, item_count, hitf, max_items, variant,
                                grid, s);
  const unsigned g = (unsigned)(max_items < grid ? max_items : grid);
  k_pass_a_valu<<<g, kBlock, 0, s>>>(d_sets, n_sets, items, item_count, hitf);
  return hipGetLastError();
}

hipError_t launch_scatter_nearest(const QuerySet* d_sets, int n_sets, hipStream_t s) {
  k_scatter_nearest<<<256, kBlock, 0, s>>>(d_sets, n_sets);
  return hipGetLastError();
}

hipError_t count_pass_b_pairs(const QuerySet* d_sets, int n_sets, const int2* items,
                              const int32_t* item_count, const unsigned char* hitf,
                              int64_t max_items, unsigned long long* h_pairs) {
  const unsigned long long zero = 0;
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(pass_b_pairs), &zero, sizeof zero, 0,
                                   hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  if (max_items > 0) {
    k_pass_b_count<<<kPersistBlocks, kBlock, 0, 0>>>(d_sets, n_sets, items, item_count, hitf);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = hipDeviceSynchronize()) != hipSuccess) return e;
  return hipMemcpyFromSymbol(h_pairs, HIP_SYMBOL(pass_b_pairs), sizeof *h_pairs, 0,
                             hipMemcpyDeviceToHost);
}

hipError_t launch_pass_b(const QuerySet* d_sets, int n_sets, const int2* items,
                         const int32_t* item_count, const unsigned char* hitf, int64_t max_items,
                         bool track_nearest, hipStream_t s) {
  if (max_items > 0) {
    const unsigned grid = (unsigned)(max_items < kPersistBlocks ? max_items : kPersistBlocks);
    if (track_nearest)
      k_pass_b<true><<<grid, kBlock, 0, s>>>(d_sets, n_sets, items, item_count, hitf);
    else
      k_pass_b<false><<<grid, kBlock, 0, s>>>(d_sets, n_sets, items, item_count, hitf);
  }
  return hipGetLastError();
}

}  // namespace aero
