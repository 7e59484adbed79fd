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

// The block's tile: R elements per thread (R kBlock per tile, chosen per call so that
// the call has enough tiles to fill the GPU), element r * kBlock + threadIdx.x of the
// tile in slice r (slices in index order, so ranks taken slice by slice keep the
// original order among equal digits).
struct Tile {
  int s;          // set
  int64_t blk;    // tile within the set
  int64_t i0;     // first element of the tile
  int n;          // elements of the tile
};

template <int R>
__device__ inline Tile locate(const SortSet* sets, int n_sets) {
  const int64_t bid = blockIdx.x;
  Tile t;
  t.s = find_owner(sets, n_sets, bid, [](const SortSet& q) { return q.block_base; });
  t.blk = bid - sets[t.s].block_base;
  t.i0 = t.blk * (R * kBlock);
  t.n = (int)min<int64_t>(R * kBlock, sets[t.s].Q - t.i0);
  return t;
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

template <int R>
__global__ __launch_bounds__(kBlock) void k_sort_hist(const SortSet* __restrict__ sets, int n_sets,
                                                      int pass, int src) {
  __shared__ int hist[kWaves][kSortDigits];
  __shared__ unsigned box[6];
  const Tile t = locate<R>(sets, n_sets);
  const SortSet& S = sets[t.s];
  for (int k = threadIdx.x; k < kWaves * kSortDigits; k += kBlock) (&hist[0][0])[k] = 0;
  // this thread's inputs, loaded before the barrier so that their latency overlaps
  // the merge of the box copies
  float p[R][3];
  uint32_t key[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = r * kBlock + threadIdx.x;
    const int64_t i = t.i0 + j;
    p[r][0] = p[r][1] = p[r][2] = 0.0f;
    key[r] = 0;
    if (j < t.n) {
      if (pass == 0) {
        const int64_t at = i * S.stride;
        p[r][0] = S.px[at];
        p[r][1] = S.py[at];
        p[r][2] = S.pz[at];
      } else {
        key[r] = S.key[src][i];
      }
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
  const int w = threadIdx.x >> 6;
  if (pass == 0) {  // the first pass also builds the keys
    AERO_GLOBAL uint32_t* __restrict__ key0 = global_ptr(S.key[0]);
    AERO_GLOBAL int32_t* __restrict__ val0 = global_ptr(S.val[0]);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int j = r * kBlock + threadIdx.x;
      if (j < t.n) {
        key[r] = morton_key(box, S.margin, p[r]);
        key0[t.i0 + j] = key[r];
        val0[t.i0 + j] = (int32_t)(t.i0 + j);
      }
    }
  }
  // the wave's digit counts over its slices (the wave's own row: no barrier needed)
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const bool on = r * kBlock + (int)threadIdx.x < t.n;
    const uint32_t dig = (key[r] >> (kSortShift0 + 8 * pass)) & 0xffu;
    int rank, count;
    wave_rank(on, dig, rank, count);
    if (on && rank == 0) hist[w][dig] += count;
  }
  __syncthreads();
  for (int d = threadIdx.x; d < kSortDigits; d += kBlock) {
    int tot = 0;
    for (int u = 0; u < kWaves; ++u) tot += hist[u][d];
    table[(int64_t)d * n_blocks + t.blk] = tot;
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

// Scatter of one pass: the tile's elements are ranked slice by slice (stable), placed
// in LDS in digit order, and written out from there, so that consecutive threads
// store consecutive addresses of a digit's run.
template <int R>
__global__ __launch_bounds__(kBlock) void k_sort_scatter(const SortSet* __restrict__ sets,
                                                         int n_sets, int pass, int src) {
  __shared__ int hist[2][kWaves][kSortDigits];  // per slice (two in flight)
  __shared__ int run[kSortDigits];   // elements of each digit in the earlier slices
  __shared__ int dstart[kSortDigits];  // first LDS slot of each digit
  __shared__ int64_t gbase[kSortDigits];  // output position of each digit's first element
  __shared__ uint32_t sk[R > 1 ? R * kBlock : 1];
  __shared__ int32_t sv[R > 1 ? R * kBlock : 1];
  __shared__ uint16_t ssrc[R > 1 ? R * kBlock : 1];  // the staged element's place in the tile
  const Tile t = locate<R>(sets, n_sets);
  const SortSet& S = sets[t.s];
  for (int k = threadIdx.x; k < 2 * kWaves * kSortDigits; k += kBlock) (&hist[0][0][0])[k] = 0;
  run[threadIdx.x] = 0;
  // this thread's keys and values, loaded before the scans so that their latency
  // overlaps them
  uint32_t key[R];
  int32_t val[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = r * kBlock + threadIdx.x;
    key[r] = j < t.n ? S.key[src][t.i0 + j] : 0u;
    val[r] = j < t.n ? S.val[src][t.i0 + j] : 0;
  }
  // digit bases: exclusive scan of the digit totals (kBlock == kSortDigits), plus the
  // tile's offset among the tiles
  int total;
  const int64_t db = block_exclusive_scan(S.rowsum[threadIdx.x], &total);
  gbase[threadIdx.x] = db + S.table[(int64_t)threadIdx.x * S.n_blocks + t.blk];
  const int w = threadIdx.x >> 6;
  int lr[R];  // rank of each element among the tile's elements of its digit
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const bool on = r * kBlock + (int)threadIdx.x < t.n;
    const uint32_t dig = (key[r] >> (kSortShift0 + 8 * pass)) & 0xffu;
    int rank, count;
    wave_rank(on, dig, rank, count);
    int(*h)[kSortDigits] = hist[r & 1];
    if (on && rank == 0) h[w][dig] = count;
    __syncthreads();  // this slice's counts (and, at r = 0, the cleared rows) are in
    int before = run[dig];
    for (int u = 0; u < w; ++u) before += h[u][dig];
    lr[r] = before + rank;
    __syncthreads();  // every lane has read run and this slice's counts
    {
      const int d = threadIdx.x;
      int add = 0;
      for (int u = 0; u < kWaves; ++u) {
        add += h[u][d];
        h[u][d] = 0;  // the row serves slice r + 2 next
      }
      run[d] += add;
    }
  }
  __syncthreads();  // run holds the tile's digit totals
  if constexpr (R > 1) {  // stage the tile in digit order
    int tt;
    dstart[threadIdx.x] = block_exclusive_scan(run[threadIdx.x], &tt);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (r * kBlock + (int)threadIdx.x >= t.n) continue;
      const uint32_t dig = (key[r] >> (kSortShift0 + 8 * pass)) & 0xffu;
      const int at = dstart[dig] + lr[r];
      sk[at] = key[r];
      sv[at] = val[r];
      ssrc[at] = (uint16_t)(r * kBlock + threadIdx.x);
    }
    __syncthreads();
  }
  // every field used below is read before the first store (a store could alias the
  // descriptor and force it to be read again behind the stores)
  AERO_GLOBAL uint32_t* __restrict__ key_out = global_ptr(S.key[1 - src]);
  AERO_GLOBAL int32_t* __restrict__ val_out = global_ptr(S.val[1 - src]);
  AERO_GLOBAL int32_t* __restrict__ inv = global_ptr(S.inv);
  AERO_GLOBAL float* __restrict__ sp = global_ptr(S.sp);
  AERO_GLOBAL float* __restrict__ tp = global_ptr(S.tp);
  float4* __restrict__ sc = S.sc;
  const float* __restrict__ px = S.px;
  const float* __restrict__ py = S.py;
  const float* __restrict__ pz = S.pz;
  const int64_t stride = S.stride;
  const int64_t Q = S.Q;
  const bool last_pass = pass == kSortPasses - 1;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = r * kBlock + threadIdx.x;
    if (j >= t.n) continue;
    // one element per thread: written from registers (a tile of one slice gains
    // nothing from staging)
    const uint32_t k = R > 1 ? sk[j] : key[r];
    const int32_t v = R > 1 ? sv[j] : val[r];
    const int64_t isrc = t.i0 + (R > 1 ? (int)ssrc[j] : j);  // the element's input place
    const uint32_t dig = (k >> (kSortShift0 + 8 * pass)) & 0xffu;
    const int64_t pos = gbase[dig] + (R > 1 ? j - dstart[dig] : lr[r]);
    if (pos < 0 || pos >= Q) continue;  // never for consistent counts; never write outside
    key_out[pos] = k;
    val_out[pos] = v;
    // the coordinates travel with the keys: read from the tile's own input (the
    // original arrays in the first pass, the first pass's output in the last), not
    // gathered through the permutation at the end
    float x, y, z;
    if (pass == 0) {
      const int64_t at = isrc * stride;
      x = px[at];
      y = py[at];
      z = pz[at];
    } else {
      x = tp[isrc];
      y = tp[Q + isrc];
      z = tp[2 * Q + isrc];
    }
    if (!last_pass) {
      tp[pos] = x;
      tp[Q + pos] = y;
      tp[2 * Q + pos] = z;
      continue;
    }
    if (v < 0 || v >= Q) continue;
    if (sc) {
      // a cloud: the points in key order with their original index
      sc[pos] = make_float4(x, y, z, __int_as_float(v));
    } else {
      // the inverse permutation, and the positions in slot order for the distance
      // passes (read there without a gather through the permutation)
      inv[v] = (int32_t)pos;
      sp[pos] = x;
      sp[Q + pos] = y;
      sp[2 * Q + pos] = z;
    }
  }
}

}  // namespace

hipError_t launch_spatial_sort(const SortSet* d_sorts, int n_sets, int64_t total_blocks,
                               int per_thread, hipStream_t s) {
  static_assert(kBlock == kSortDigits, "one thread per digit in the scans");
  static_assert(kSortPasses == 2, "the coordinates go original -> tp -> the output");
  if (total_blocks <= 0 || n_sets <= 0) return hipSuccess;
  const unsigned g = (unsigned)total_blocks;
  int src = 0;
  for (int pass = 0; pass < kSortPasses; ++pass) {
    switch (per_thread) {
      case 8: k_sort_hist<8><<<g, kBlock, 0, s>>>(d_sorts, n_sets, pass, src); break;
      case 4: k_sort_hist<4><<<g, kBlock, 0, s>>>(d_sorts, n_sets, pass, src); break;
      case 2: k_sort_hist<2><<<g, kBlock, 0, s>>>(d_sorts, n_sets, pass, src); break;
      default: k_sort_hist<1><<<g, kBlock, 0, s>>>(d_sorts, n_sets, pass, src); break;
    }
    k_sort_rowscan<<<(unsigned)(n_sets * kSortDigits), kBlock, 0, s>>>(d_sorts);
    switch (per_thread) {
      case 8: k_sort_scatter<8><<<g, kBlock, 0, s>>>(d_sorts, n_sets, pass, src); break;
      case 4: k_sort_scatter<4><<<g, kBlock, 0, s>>>(d_sorts, n_sets, pass, src); break;
      case 2: k_sort_scatter<2><<<g, kBlock, 0, s>>>(d_sorts, n_sets, pass, src); break;
      default: k_sort_scatter<1><<<g, kBlock, 0, s>>>(d_sorts, n_sets, pass, src); break;
    }
    src = 1 - src;
  }
  return hipGetLastError();
}

}  // namespace aero
