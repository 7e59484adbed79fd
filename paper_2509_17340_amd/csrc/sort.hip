// Spatial sort of the rollout positions before the first distance pass (the
// positions' bounding box is merged by the rollout kernel as it writes them), and of
// the cloud in the same launches.
//
// The first pass takes blocks of consecutive positions; its per-block bound and the
// cloud sub-tiles a block comes near are only as tight as the block is compact.
// Positions of one (instance, step) are spread by the sampling noise, so they are
// reordered along a Morton (Z-order) curve over their bounding box: a stable LSD
// radix sort on the top 16 bits of a 24-bit key (8 bits per axis), in two passes of
// 8 bits (cells of 1/32 of the box per axis; within a cell the original order is
// kept).  The cloud is keyed on the same box widened by a margin, so that its points
// near the positions fall into compact sub-tiles; a cloud made of several
// accumulated sweeps is far less compact in its given order.
// Every pass ranks elements without atomics (ballots inside a wave, per-wave counts
// in LDS, per-block counts scanned in digit-major order), so the permutation is
// deterministic and the same for a problem alone or inside a batch.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "aero_device.h"
#include "aero_internal.h"

namespace aero {
namespace {

constexpr int kWaves = kBlock / 64;
constexpr int kSortShift0 = 8;  // the key's lowest 8 bits are not sorted on

// Inverse of ord_bits: the float whose order-preserving bits are o.
__device__ inline float ord_float(unsigned o) {
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

// The low 10 bits of v moved to every third bit.
__device__ inline uint32_t spread3(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

struct Elem {
  int s;          // set
  int64_t blk;    // block within the set
  int64_t i;      // element within the set
  bool active;
};

__device__ inline Elem locate(const SortSet* sets, int n_sets) {
  const int64_t bid = blockIdx.x;
  Elem e;
  e.s = find_owner(sets, n_sets, bid, [](const SortSet& q) { return q.block_base; });
  e.blk = bid - sets[e.s].block_base;
  e.i = e.blk * kBlock + threadIdx.x;
  e.active = e.i < sets[e.s].Q;
  return e;
}

// Morton key of an element from its position and the key box (the set's bounding
// box widened by `margin`; positions outside it are clamped to its boundary cells).
// box: the positions' bounding box (order-preserving bits), merged from the rollout's
// copies by the first pass.
__device__ inline uint32_t morton_key(const unsigned box[6], float margin, const float p[3]) {
  float lo[3], ext = 0.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = ord_float(box[a]) - margin;
    ext = fmaxf(ext, (ord_float(box[3 + a]) + margin) - lo[a]);
  }
  const float scale = ext > 0.0f ? 255.99f / ext : 0.0f;
  uint32_t key = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float g = fminf(fmaxf((p[a] - lo[a]) * scale, 0.0f), 255.0f);
    key |= spread3((uint32_t)g) << a;
  }
  return key;
}

// Rank of this lane's digit among the equal digits of lower lanes, and how many
// lanes of the wave hold it (only active lanes take part).
__device__ inline void wave_rank(bool active, uint32_t dig, int& rank, int& count) {
  uint64_t match = __ballot(active);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (dig >> b) & 1u;
    const uint64_t m = __ballot(bit);
    match &= bit ? m : ~m;
  }
  const int lane = threadIdx.x & 63;
  rank = __popcll(match & ((1ull << lane) - 1ull));
  count = __popcll(match);
}

__global__ __launch_bounds__(kBlock) void k_sort_hist(const SortSet* __restrict__ sets, int n_sets,
                                                      int pass, int src) {
  __shared__ int hist[kWaves][kSortDigits];
  __shared__ unsigned box[6];
  const Elem e = locate(sets, n_sets);
  const SortSet& S = sets[e.s];
  for (int k = threadIdx.x; k < kWaves * kSortDigits; k += kBlock) (&hist[0][0])[k] = 0;
  // this element's input, loaded before the barrier so that its latency overlaps the
  // merge of the box copies
  float p[3] = {0.0f, 0.0f, 0.0f};
  uint32_t key = 0;
  if (e.active) {
    if (pass == 0) {
      const int64_t at = e.i * S.stride;
      p[0] = S.px[at];
      p[1] = S.py[at];
      p[2] = S.pz[at];
    } else {
      key = S.key[src][e.i];
    }
  }
  if (pass == 0 && threadIdx.x < 6) {  // merge the box copies (minima, then maxima)
    const int a = threadIdx.x;
    unsigned v = S.box[a];
    for (int cp = 1; cp < kBoxCopies; ++cp) {
      const unsigned w = S.box[cp * kBoxStride + a];
      v = a < 3 ? min(v, w) : max(v, w);
    }
    box[a] = v;
  }
  __syncthreads();
  AERO_GLOBAL int32_t* __restrict__ table = global_ptr(S.table);
  const int64_t n_blocks = S.n_blocks;
  if (e.active && pass == 0) {  // the first pass also builds the keys
    key = morton_key(box, S.margin, p);
    AERO_GLOBAL uint32_t* __restrict__ key0 = global_ptr(S.key[0]);
    AERO_GLOBAL int32_t* __restrict__ val0 = global_ptr(S.val[0]);
    key0[e.i] = key;
    val0[e.i] = (int32_t)e.i;
  }
  const uint32_t dig = (key >> (kSortShift0 + 8 * pass)) & 0xffu;
  int rank, count;
  wave_rank(e.active, dig, rank, count);
  if (e.active && rank == 0) hist[threadIdx.x >> 6][dig] = count;
  __syncthreads();
  for (int d = threadIdx.x; d < kSortDigits; d += kBlock) {
    int tot = 0;
    for (int w = 0; w < kWaves; ++w) tot += hist[w][d];
    table[(int64_t)d * n_blocks + e.blk] = tot;
  }
}

// Exclusive scan of v over the block's kBlock threads; *total receives the sum.
__device__ inline int block_exclusive_scan(int v, int* total) {
  __shared__ int wsum[kWaves];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int before = 0, all = 0;
  for (int k = 0; k < kWaves; ++k) {
    if (k < w) before += wsum[k];
    all += wsum[k];
  }
  __syncthreads();
  *total = all;
  return before + x - v;
}

// One block per (set, digit): exclusive scan of that digit's per-block counts.
__global__ __launch_bounds__(kBlock) void k_sort_rowscan(const SortSet* __restrict__ sets) {
  const int s = blockIdx.x / kSortDigits, d = blockIdx.x % kSortDigits;
  const SortSet& S = sets[s];
  if (S.n_blocks == 0) return;  // block-uniform: a set without positions to sort
  int32_t* row = S.table + (int64_t)d * S.n_blocks;
  const int n = S.n_blocks;
  const int per = (n + kBlock - 1) / kBlock;
  const int b0 = min(n, (int)threadIdx.x * per), b1 = min(n, b0 + per);
  int sum = 0;
  for (int b = b0; b < b1; ++b) sum += row[b];
  int total;
  int run = block_exclusive_scan(sum, &total);
  for (int b = b0; b < b1; ++b) {
    const int c = row[b];
    row[b] = run;
    run += c;
  }
  if (threadIdx.x == 0) S.rowsum[d] = total;
}

__global__ __launch_bounds__(kBlock) void k_sort_scatter(const SortSet* __restrict__ sets,
                                                         int n_sets, int pass, int src) {
  __shared__ int hist[kWaves][kSortDigits];
  __shared__ int base[kSortDigits];
  const Elem e = locate(sets, n_sets);
  const SortSet& S = sets[e.s];
  for (int k = threadIdx.x; k < kWaves * kSortDigits; k += kBlock) (&hist[0][0])[k] = 0;
  // this element's key and value, loaded before the scan so that their latency
  // overlaps it
  const uint32_t k = e.active ? S.key[src][e.i] : 0u;
  const int32_t v = e.active ? S.val[src][e.i] : 0;
  // digit bases: exclusive scan of the digit totals (kBlock == kSortDigits)
  int total;
  base[threadIdx.x] = block_exclusive_scan(S.rowsum[threadIdx.x], &total);
  __syncthreads();
  const uint32_t dig = (k >> (kSortShift0 + 8 * pass)) & 0xffu;
  int rank, count;
  wave_rank(e.active, dig, rank, count);
  const int w = threadIdx.x >> 6;
  if (e.active && rank == 0) hist[w][dig] = count;
  __syncthreads();
  if (e.active) {
    int before = 0;
    for (int u = 0; u < w; ++u) before += hist[u][dig];
    const int64_t pos = (int64_t)base[dig] + S.table[(int64_t)dig * S.n_blocks + e.blk] + before +
                        rank;
    const int64_t Q = S.Q;
    if (pos >= 0 && pos < Q) {  // always true for consistent counts; never write outside
      // every field used below is read before the first store (a store could alias
      // the descriptor and force it to be read again behind the stores)
      AERO_GLOBAL uint32_t* __restrict__ key_out = global_ptr(S.key[1 - src]);
      AERO_GLOBAL int32_t* __restrict__ val_out = global_ptr(S.val[1 - src]);
      const bool last = pass == kSortPasses - 1 && v >= 0 && v < Q;
      AERO_GLOBAL int32_t* __restrict__ inv = global_ptr(S.inv);
      AERO_GLOBAL float* __restrict__ sp = global_ptr(S.sp);
      float4* __restrict__ sc = S.sc;
      float p[3] = {0.0f, 0.0f, 0.0f};
      if (last) {
        const int64_t at = (int64_t)v * S.stride;
        p[0] = S.px[at];
        p[1] = S.py[at];
        p[2] = S.pz[at];
      }
      key_out[pos] = k;
      val_out[pos] = v;
      if (last && sc) {
        // a cloud: the points in key order with their original index
        sc[pos] = make_float4(p[0], p[1], p[2], __int_as_float(v));
      } else if (last) {
        // the inverse permutation, and the positions in slot order for the
        // distance passes (read there without a gather through the permutation)
        inv[v] = (int32_t)pos;
        sp[pos] = p[0];
        sp[Q + pos] = p[1];
        sp[2 * Q + pos] = p[2];
      }
    }
  }
}

}  // namespace

hipError_t launch_spatial_sort(const SortSet* d_sorts, int n_sets, int64_t total_blocks,
                               hipStream_t s) {
  static_assert(kBlock == kSortDigits, "one thread per digit in the scans");
  if (total_blocks <= 0 || n_sets <= 0) return hipSuccess;
  const unsigned g = (unsigned)total_blocks;
  int src = 0;
  for (int pass = 0; pass < kSortPasses; ++pass) {
    k_sort_hist<<<g, kBlock, 0, s>>>(d_sorts, n_sets, pass, src);
    k_sort_rowscan<<<(unsigned)(n_sets * kSortDigits), kBlock, 0, s>>>(d_sorts);
    k_sort_scatter<<<g, kBlock, 0, s>>>(d_sorts, n_sets, pass, src);
    src = 1 - src;
  }
  return hipGetLastError();
}

}  // namespace aero
