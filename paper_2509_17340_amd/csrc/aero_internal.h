// Host/device shared layout of the AERO-MPPI library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/aero.h"

namespace aero {

#ifndef AERO_TILE_PTS
#define AERO_TILE_PTS 1024
#endif
#ifndef AERO_QUERIES_PER_LANE
#define AERO_QUERIES_PER_LANE 8
#endif

constexpr int kBlock = 256;                              // threads per workgroup (4 wave64)
constexpr int kTilePts = AERO_TILE_PTS;                  // cloud points per tile (box hierarchy)
constexpr int kSelCopies = 8;                            // Stage-II distance copies (atomics spread)
// The rollout's waves merge their position bounds into kBoxCopies copies of the sort
// box (a wave's copy is its workgroup index modulo kBoxCopies), each in a 256-byte
// line of its own, so that hundreds of waves do not meet on one word; the sort
// merges the copies.
constexpr int kBoxCopies = 16;
constexpr int kBoxStride = 64;  // words per copy
constexpr int kTileSplit = 4;                            // sub-tiles per tile
constexpr int kSubPts = kTilePts / kTileSplit;           // cloud points per sub-tile (work unit)
constexpr int kGroupsPerSub = kSubPts / 32;              // 32-point groups per sub-tile
constexpr int kSuperTiles = 16;                          // tiles per super-tile (cull step)
constexpr int kQueriesPerLane = AERO_QUERIES_PER_LANE;   // positions in registers per lane
constexpr int kQueriesPerBlock = kBlock * kQueriesPerLane;
static_assert(kSubPts == kBlock, "a sub-tile is staged one point per thread");

// Pass-A variants (the expanded-form first pass of the distance computation).  Each
// runs over the (query block, cloud sub-tile) pairs that the cull step lists.
constexpr int kPassAValu = 0;    // VALU FMAs, kQueriesPerBlock positions per block
constexpr int kPassAF16s4 = 1;   // half-precision matrix cores on split coordinates,
                                 //   4 column blocks of 32 per wave: 512 per block
constexpr int kPassAF16s8 = 2;   //   the same with 8 column blocks: 1024 per block
constexpr int kPassAVariants = 3;
constexpr int kPassAQPB[kPassAVariants] = {kQueriesPerBlock, 4 * 32 * 4, 4 * 32 * 8};
constexpr int kPassAMinQPB = 4 * 32 * 4;
// Launch configurations the autotuner chooses among: a pass-A variant and the number
// of persistent workgroups it runs with.  Configuration v < kPassAVariants is variant
// v at its default grid (a forced variant runs that).
struct PassAConfig {
  int variant;
  int grid;
};
constexpr int kPassAConfigs = 5;
constexpr PassAConfig kPassAConf[kPassAConfigs] = {
    {kPassAValu, 1024}, {kPassAF16s4, 4096}, {kPassAF16s8, 4096},
    {kPassAF16s4, 1024}, {kPassAF16s8, 1024}};
// Pass B gives each lane at most kQueriesPerLane queries of one pass-A block.
static_assert(kQueriesPerBlock <= kQueriesPerLane * kBlock && kPassAMinQPB <= kQueriesPerBlock &&
                  4 * 32 * 8 <= kQueriesPerBlock, "pass-A blocks must fit one pass-B block");

// Per-problem record, built on the host and copied into the workspace.
struct DevProblem {
  const float* cloud;
  int32_t n_points, M, K, N;
  uint32_t problem_id, pad0;
  float x0[10];
  float pg[3], vg[3], qg[4];
  const float* coef;     // [M][3][6]
  float* u_nom;          // [M][N][4]
  double* S1;            // [M][K]
  double* J_ctrl;        // [M][K]  control term, written by the rollout
  float* state;          // [M][N][K][10] state after every step (p, q, v) rounded to
                         //   float32, written by the rollout and scored by the finalize
                         //   kernel
  float* deff;           // [M][N][4][K]
  float* pos;            // [3][M][N][K] planes x, y, z
  unsigned* mind2;       // [M][N][K] float bits of the squared nearest distance
  int64_t sample_base;   // prefix of M*K over problems
  int64_t row_base;      // prefix of M*N over problems
  double* J;             // optional [5][M*K] unweighted terms (track, vnorm, ctrl, goal, col)
  int32_t* nidx;         // optional [M][N][K] nearest point index (-1: none within reach)
  int32_t* item_count;   // the call's (query block, sub-tile) item counter (or nullptr)
  unsigned* sort_box;    // [kBoxCopies][kBoxStride] copies of the position bounding box
                         //   of the spatial sort (or nullptr)
  double* noise;         // [M][N][4][K] standard normals drawn ahead of the rollout
  unsigned* out_slot;    // sorted query set's distances by slot (or nullptr)
  const int32_t* inv;    // sorted query set: query -> slot (or nullptr: distances in mind2)
  const int32_t* nidx_in;  // nearest indices given by the caller (indexed adjoint)
  int64_t elem_base;     // prefix of M*N*K over problems
  const float* w_dev;    // optional [5] device term weights replacing DevParams::w
  unsigned long long* nn;  // the set's pass-B nearest records by slot (reset with the
                           //   distances), or nullptr
  unsigned* amin;          // the set's least pass-A values by slot (reset with the
                           //   distances), or nullptr
  int64_t inst_base;       // prefix of M over problems
  double* wexp;            // [M][K] e_k = exp(-(S1_k - rho) / lambda) of each instance
  double* eta;             // [M] sum_k e_k
};

// Spatial sort of one problem's rollout positions, or of its cloud (stable LSD radix
// sort on the top 16 bits of a 24-bit Morton key, 2 passes of 8 bits).  Both key on the
// positions' bounding box (the cloud's box widened by `margin`, so that cloud points
// near the positions get fine cells and the far ones collect in boundary cells).
constexpr int kSortDigits = 256;
constexpr int kSortPasses = 2;
// Elements per thread of a sort workgroup (1, 2, 4 or 8; tiles of that many times
// kBlock): the most that still leaves the call about kSortMinGrid tiles.
constexpr int kSortMaxPerThread = 8;
constexpr int64_t kSortMinGrid = 1024;
struct SortSet {
  const float* px;       // element i at px[i * stride] (planes: stride 1; cloud: stride 3)
  const float* py;
  const float* pz;
  float* sp;             // positions: [3][Q] in slot order (written by the last pass)
  float* tp;             // [3][Q] the coordinates in the first pass's output order
  int64_t Q;
  int64_t block_base;    // prefix of n_blocks over sets
  int32_t n_blocks;      // ceil(Q / tile), tile = kBlock x the call's elements per thread
  int32_t stride;
  unsigned* box;         // [kBoxCopies][kBoxStride] copies; words 0..5 of each hold the
                         //   order-preserving bits of min x, y, z, max x, y, z
  uint32_t* key[2];      // [Q] ping-pong keys
  int32_t* val[2];       // [Q] ping-pong element indices; the result is
                         //   val[kSortPasses % 2]
  int32_t* inv;          // positions: [Q] query -> slot (written by the last pass)
  int32_t* table;        // [kSortDigits][n_blocks] per-block digit counts -> offsets
  int32_t* rowsum;       // [kSortDigits] digit totals
  float4* sc;            // cloud: [Q] sorted points (x, y, z, original index as int bits)
  float margin;          // key box = box widened by margin on every side
  int32_t pad;
};

// One set of query positions scored against one cloud by the distance kernels.
//
// Exact sets (items == nullptr) run the direct-form kernel over every query against
// the cloud tiles within d_max of its wave's queries.  Two-pass sets are cut into
// query blocks of qpbA consecutive (spatially sorted) positions.  The cull step gives
// each block a centre, a bound on its pass-A rounding error, and the list of cloud
// sub-tiles whose bounding box lies within reach of the block's box, in the raw or
// the sorted cloud order (whichever lists fewer); pass A runs the recentred expanded
// form over those (block, sub-tile) items only and records, per item, which of the
// block's queries came under the bound there; pass B reruns the direct form for
// exactly those (query, sub-tile) pairs.
struct QuerySet {
  const float* px;
  const float* py;
  const float* pz;
  const float* sp;       // [3][Q] positions in slot order (planes x, y, z): the spatial
                         //   sort's output for sorted sets, else px itself
  unsigned* out;         // min squared distance as float bits, pre-filled with +inf;
                         //   exact sets: n_copies arrays of Q, merged by their reader
  const float* cloud;    // [n_points][3]
  int64_t Q;             // queries
  int32_t n_copies;      // exact sets: copies of `out` that workgroups spread their
                         //   atomics over (workgroup b uses copy b % n_copies)
  int32_t n_points;
  int32_t n_qblocks;     // ceil(Q / qpbA)
  int32_t n_chunks;      // exact sets: cloud splits, chunk c covers points
  int32_t chunk_pts;     //   [c chunk_pts, min((c+1) chunk_pts, n_points))
  int32_t qpbA;          // positions per query block
  int64_t block_base;    // exact sets: prefix of n_qblocks * n_chunks over sets
  // two-pass extension
  float4* binfo;         // [n_qblocks] block centre (x, y, z) and flag bound (w) on the
                         //   pass-A squared distance
  float* tbox;           // [n_tiles][6] tile bounding boxes (lo, hi) of the raw cloud
  float* sbox;           // [n_sub][6] sub-tile bounding boxes of the raw cloud
  float* gbox;           // [n_sub * kGroupsPerSub][6] boxes of their 32-point groups
  const float4* scloud;  // [n_points] the cloud in Morton order (x, y, z, original
                         //   index bits), or nullptr: raw order only
  float* stbox;          // [n_tiles][6], [n_sub][6], [n_sub * kGroupsPerSub][6]: boxes
  float* ssbox;          //   of the sorted cloud
  float* sgbox;
  float* ubox;           // [ceil(n_tiles / kSuperTiles)][6] boxes of kSuperTiles
  float* subox;          //   consecutive tiles, raw and sorted cloud (cull step)
  int2* items;           // the call's item list: (global query block, sub-tile | order
                         //   << 31); a block's items are consecutive
  int32_t* item_count;   // entries of `items` (zeroed by the noise kernel)
  unsigned char* hitf;   // [items]: 1 where some query of the block came under the bound
  uint32_t* hmask;       // the call's hit words: item i's qpbA bits at i * (qpbA / 32)
                         //   (bit j of word w: query w * 32 + j of the block came under
                         //   the bound in the item's sub-tile), for the items with
                         //   (i + 1) * qpbA / 32 <= mask_words; pass B takes every
                         //   query of the block for a marked item beyond that
  int64_t mask_words;
  int64_t qb_base;       // prefix of n_qblocks over two-pass sets (global block index)
  int64_t tile_base;     // prefix of n_tiles over two-pass sets
  int64_t query_base;    // prefix of ceil(Q / kBlock) flag blocks over sets
  int32_t n_tiles;       // ceil(n_points / kTilePts)
  int32_t cull;          // 0: every sub-tile of the raw cloud is listed (brute force)
  float d_max;
  int32_t pad1;
  const int32_t* perm;   // [Q] slot -> query, spatially sorted (nullptr: identity)
  unsigned* out_slot;    // two-pass sets: [Q] squared distances by slot (== out without
                         //   a sort), exact where pass B evaluated some pair of the
                         //   query, +inf elsewhere (no point within d_max); read back to
                         //   `out` by the finalize kernel
  unsigned long long* nn;  // optional [Q]: pass B also keeps (d^2 bits << 32 | index) per
                           // slot (lowest index on ties)
  int32_t* nidx;           // with nn: [Q] nearest index per query (-1: none evaluated)
  unsigned* amin;          // two-pass sets: [Q] by slot, the least pass-A value of each
                           //   query over the items where it came under the bound (float
                           //   bits, clamped at 0; +inf elsewhere): with the block's
                           //   bound it caps the query's nearest squared distance, so
                           //   pass B skips point groups beyond that cap
};

// One planning problem's front end (partition, anchors, guides) as the batched
// front-end kernels read it; built on the host from aero_front_end_job.
struct FrontJob {
  const float* tables;      // direction tables of the fine grid (aero_partition_tables)
  const float* cloud;       // [n_points][3]
  unsigned long long* key;  // [n_fine] binary64 bits of the cone minima
  unsigned* idx;            // [n_fine] lowest point index attaining them
  int32_t* coarse_best;     // [n_coarse]
  int32_t* anchor_cell;     // [M]
  int32_t* anchor_fine;     // [M]
  float* anchors;           // [M][3]
  float* coef;              // [M][3][6] guide coefficients
  const float* end_vel;     // optional [M][3]
  const float* end_acc;     // optional [M][3]
  int64_t cell_base;        // prefix of fine cells over jobs
  int64_t block_base;       // prefix of point blocks (kBlock points) over jobs
  int32_t n_points, n_az_c, n_el_c, f_a, f_e, M_h, M_v, pad;
  float r_max, ell, T, pad1;
  float p0[3], goal[3], v0[3], a0[3];
};

// Parameters promoted once on the host.
struct DevParams {
  double dt, lambda, mass, gravity;
  double sigma[4], u_min[4], u_max[4];
  double Q_track, Q_vnorm, Q_c, Q_cdelta, Q_p, Q_v, Q_q, C, a, d_min, d_max;
  double w[5];
  uint32_t seed_lo, seed_hi, iter_base, pad;
};

// Query of pass-A slot `slot` (a permutation of [0, Q); clamped, so that even a
// corrupt permutation cannot address outside the positions).
__device__ inline int64_t perm_query(const QuerySet& S, int64_t slot) {
  if (!S.perm) return slot;
  const int64_t q = S.perm[slot];
  return q < 0 ? 0 : (q >= S.Q ? S.Q - 1 : q);
}

// Squared distance between two axis-aligned boxes (0 when they overlap).  Monotone:
// a box containing another is never farther.
__device__ __forceinline__ float box_dist2(const float* b, const float lo[3], const float hi[3]) {
  float d2 = 0.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float dd = fmaxf(0.0f, fmaxf(b[a] - hi[a], lo[a] - b[3 + a]));
    d2 = fmaf(dd, dd, d2);
  }
  return d2;
}

// Squared reach of a query block with pass-A bound thr: pass A errs by at most
// thr - d_max^2 on every pair within d_max, so every point within d_max of a query, and
// every point whose pass-A value falls below thr, lies within r2 = 2 thr - d_max^2 of
// it, hence its sub-tile's box within r2 of the block's box.  The relative margin
// covers the rounding of the box distance.
__device__ inline float reach_limit(float thr, float d_max) {
  const float r2 = thr < INFINITY ? thr + (thr - d_max * d_max) : INFINITY;
  return r2 * (1.0f + 1e-5f) + 1e-6f;
}

// Per-problem Stage-II record.
struct DevSelect {
  const float* cloud;
  int32_t n_points, M, N, pad0;
  float x0[10];
  float pg[3], vg[3], qg[4];
  const float* u_nom;    // [M][N][4]
  double* state;         // [M][N][10] states of the noise-free rollouts
  float* pos;            // [3][M][N]
  unsigned* mind2;       // [kSelCopies][M][N] partial minima, merged by k_sel_final
  double* S2;            // [M] (caller's array + offset)
  int32_t* best;         // caller's array + problem index
  int64_t inst_base;     // prefix of M
  const float* w_dev;    // optional [5] device term weights replacing DevParams::w
};

// The term weights of a problem: its device weights when given, else the call's.
__device__ inline void load_weights(const float* w_dev, DevParams& prm) {
  if (w_dev)
    for (int i = 0; i < 5; ++i) prm.w[i] = (double)w_dev[i];
}

// Kernel launchers (defined in the .hip files).
hipError_t launch_put_bytes(void* dst, const void* src, size_t bytes, hipStream_t s);
hipError_t launch_spatial_sort(const SortSet* d_sorts, int n_sets, int64_t total_blocks,
                               int per_thread, hipStream_t s);
hipError_t launch_accumulate_cloud(const float* ring, int64_t ring_points, const int32_t* start,
                                   const int32_t* offsets, int F, int64_t n_points,
                                   const float* poses, const float* origin, float* out,
                                   hipStream_t s);
hipError_t launch_advance_state(const float* x0, const float* u, int M, int N,
                                const int32_t* index, const DevParams& prm, float* x1,
                                hipStream_t s);
hipError_t launch_shift_controls(const float* src, int M_src, int N, const int32_t* index,
                                 int shift, float* dst, int M_dst, hipStream_t s);
hipError_t launch_step_candidates(const float* u, const float* g, int N, float s0, float beta,
                                  int n, const DevParams& prm, float* out, hipStream_t s);
hipError_t launch_partition(const aero_partition_spec& spec, const float* cloud, int n_points,
                            const float goal[3], double* fine_key, int32_t* fine_idx,
                            int32_t* coarse_best, int32_t* anchor_cell, int32_t* anchor_fine,
                            float* anchors, hipStream_t s);
hipError_t launch_filter_cloud(const float* cloud, int n_points, const int32_t* fine_idx,
                               int n_fine, float* out, hipStream_t s);
// Partition, anchors and guides of n jobs in three launches (descriptors carried in
// the first launch's argument when they fit, else uploaded to d_jobs first).
hipError_t launch_front_end(FrontJob* d_jobs, const FrontJob* h_jobs, int n, int64_t total_cells,
                            int64_t total_blocks, hipStream_t s);
hipError_t launch_guides(const double p0[3], const double v0[3], const double a0[3],
                         const float* anchors, const float* end_vel, const float* end_acc,
                         double T, int M, float* coef, hipStream_t s);
hipError_t launch_rollout_noise(const DevProblem* d_probs, int n, int64_t total_samples,
                                int64_t total_elems, const DevParams& prm, const QuerySet* d_sets,
                                int64_t box_blocks, const void* h_blob, size_t blob_bytes,
                                hipStream_t s);
hipError_t launch_sorted_boxes(const QuerySet* d_sets, int n_sets, int64_t total_tiles,
                               hipStream_t s);
hipError_t launch_cull(const QuerySet* d_sets, int n_sets, int64_t total_qblocks, int variant,
                       hipStream_t s);
hipError_t launch_rollout(const DevProblem* d_probs, int n, int64_t total_samples,
                          const DevParams& prm, hipStream_t s);
hipError_t launch_min_dist(const QuerySet* d_sets, int n_sets, int64_t total_blocks,
                           float d_max, hipStream_t s);
// The first pass over the call's item list (items, item_count and hitf are shared by
// every two-pass set of the call); max_items bounds the list (the grid is sized by it).
hipError_t launch_pass_a(const QuerySet* d_sets, int n_sets, const int2* items,
                         const int32_t* item_count, unsigned char* hitf, int64_t max_items,
                         int variant, int grid, hipStream_t s);
hipError_t launch_pass_a_matrix(const QuerySet* d_sets, int n_sets, const int2* items,
                                const int32_t* item_count, unsigned char* hitf, int64_t max_items,
                                int variant, int grid, hipStream_t s);
// Pass B over the marked items (the hit words of every set of the call share one array);
// track_nearest: some set keeps nearest indices (nn).
// Pairs pass A evaluates on the items of the last call: h_pairs[0] existing positions x
// points of the groups taken, h_pairs[1] matrix-core product pairs (synchronous, null
// stream).
hipError_t count_pass_a_pairs(const QuerySet* d_sets, int n_sets, const int2* items,
                              const int32_t* item_count, int64_t max_items,
                              unsigned long long* h_pairs);
// Pairs pass B evaluates on the items of the last call (synchronous, null stream).
hipError_t count_pass_b_pairs(const QuerySet* d_sets, int n_sets, const int2* items,
                              const int32_t* item_count, const unsigned char* hitf,
                              int64_t max_items, unsigned long long* h_pairs);
hipError_t launch_pass_b(const QuerySet* d_sets, int n_sets, const int2* items,
                         const int32_t* item_count, const unsigned char* hitf, int64_t max_items,
                         bool track_nearest, hipStream_t s);
hipError_t launch_scatter_nearest(const QuerySet* d_sets, int n, hipStream_t s);
hipError_t launch_adjoint(const DevProblem* d_prob, const DevParams& prm, int64_t samples,
                          double* ckpt, double* seg, double* gsamp, hipStream_t s);
hipError_t launch_grad_reduce(const DevProblem* d_prob, const DevParams& prm, int64_t rows,
                              const double* gsamp, const float* grad_L, float* grad_u,
                              float* grad_w, double* wpart, hipStream_t s);
size_t grad_w_parts();  // doubles of the weight-gradient partial sums
hipError_t launch_finalize(const DevProblem* d_probs, int n, int64_t total_samples,
                           const DevParams& prm, bool write_s1, hipStream_t s);
// The control update: per instance the weights (rho, e_k, eta), then per (instance,
// step) row the weighted perturbation sum.
hipError_t launch_update(const DevProblem* d_probs, int n, int64_t total_inst, int64_t total_rows,
                         const DevParams& prm, hipStream_t s);
hipError_t launch_select_rollout(const DevSelect* d_sel, int n, int64_t total_inst,
                                 const DevParams& prm, const void* h_blob, size_t blob_bytes,
                                 hipStream_t s);
hipError_t launch_select_final(const DevSelect* d_sel, int n, const DevParams& prm,
                               hipStream_t s);

}  // namespace aero
