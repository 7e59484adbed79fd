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
#ifndef AERO_F16_COLS
#define AERO_F16_COLS 8
#endif

constexpr int kBlock = 256;                              // threads per workgroup (4 wave64)
constexpr int kTilePts = AERO_TILE_PTS;                  // cloud points staged in LDS per tile
constexpr int kSelCopies = 8;                            // Stage-II distance copies (atomics spread)
// The rollout's waves merge their position bounds into kBoxCopies copies of the sort
// box (a wave's copy is its workgroup index modulo kBoxCopies), each in a 256-byte
// line of its own, so that hundreds of waves do not meet on one word; the sort
// merges the copies.
constexpr int kBoxCopies = 16;
constexpr int kBoxStride = 64;  // words per copy
constexpr int kTileSplit = 4;                            // sub-tiles per tile (pass-B work units)
constexpr int kSubPts = kTilePts / kTileSplit;           // cloud points per sub-tile
constexpr int kQueriesPerLane = AERO_QUERIES_PER_LANE;   // positions in registers per lane
constexpr int kQueriesPerBlock = kBlock * kQueriesPerLane;

// Pass-A variants (the expanded-form first pass of the distance computation).
constexpr int kPassAValu = 0;   // VALU FMAs, kQueriesPerBlock positions per block
constexpr int kPassAMfma = 1;   // matrix-core MFMA, 512 positions per block
constexpr int kPassAF16s = 2;   // half-precision matrix cores on split coordinates, 1024 per block
constexpr int kPassAVariants = 3;
constexpr int kF16Cols = AERO_F16_COLS;   // split-f16 pass A: column blocks of 32 queries per wave
constexpr int kPassAQPB[kPassAVariants] = {kQueriesPerBlock, 512, 4 * 32 * kF16Cols};
// Pass B gives each lane at most kQueriesPerLane queries of one pass-A block.
static_assert(kTileSplit <= 4, "sub-tile masks take the low 4 bits of a work entry");
static_assert(kQueriesPerBlock <= kQueriesPerLane * kBlock && 512 <= kQueriesPerBlock &&
                  4 * 32 * kF16Cols <= kQueriesPerBlock, "pass-A blocks must fit one pass-B block");

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
  double* state;         // [M][N][K][10] state after every step (p, q, v), written by the
                         //   rollout and scored by the finalize kernel
  float* deff;           // [M][N][4][K]
  float* pos;            // [3][M][N][K] planes x, y, z
  unsigned* mind2;       // [M][N][K] float bits of the squared nearest distance
  int64_t sample_base;   // prefix of M*K over problems
  int64_t row_base;      // prefix of M*N over problems
  double* J;             // optional [5][M*K] unweighted terms (track, vnorm, ctrl, goal, col)
  int32_t* nidx;         // optional [M][N][K] nearest point index (-1: none within reach)
  int32_t* work_count;   // pass-B work counter of the problem's query set (or nullptr)
  unsigned* sort_box;    // [kBoxCopies][kBoxStride] copies of the position bounding box
                         //   of the spatial sort (or nullptr)
  double* noise;         // [M][N][4][K] standard normals drawn ahead of the rollout
  unsigned* out_slot;    // sorted query set's distances by slot (or nullptr)
  const int32_t* inv;    // sorted query set: query -> slot (or nullptr: distances in mind2)
  const int32_t* nidx_in;  // nearest indices given by the caller (indexed adjoint)
  int64_t elem_base;     // prefix of M*N*K over problems
  const float* w_dev;    // optional [5] device term weights replacing DevParams::w
};

// Spatial sort of one problem's rollout positions (stable LSD radix sort on the top
// 16 bits of a 24-bit Morton key over the positions' bounding box, 2 passes of 8 bits).
constexpr int kSortDigits = 256;
constexpr int kSortPasses = 2;
struct SortSet {
  const float* px;
  const float* py;
  const float* pz;
  float* sp;             // [3][Q] positions in slot order (written by the last pass)
  int64_t Q;
  int64_t block_base;    // prefix of n_blocks over sets
  int32_t n_blocks;      // ceil(Q / kBlock)
  int32_t pad;
  unsigned* box;         // [kBoxCopies][kBoxStride] copies; words 0..5 of each hold the
                         //   order-preserving bits of min x, y, z, max x, y, z
  uint32_t* key[2];      // [Q] ping-pong keys
  int32_t* val[2];       // [Q] ping-pong query indices; the result is
                         //   val[kSortPasses % 2]
  int32_t* inv;          // [Q] query -> slot (written by the last pass)
  int32_t* table;        // [kSortDigits][n_blocks] per-block digit counts -> offsets
  int32_t* rowsum;       // [kSortDigits] digit totals
};

// One set of query positions scored against one cloud by the distance kernels.
//
// Exact sets (list == nullptr) run the direct-form kernel over every query.
// Two-pass sets run the recentred expanded form over every query (pass A), flag
// the queries whose approximate squared distance is below a per-block bound
// (`thresh`, derived from the rounding error of pass A), and rerun the direct
// form on the flagged list only (pass B).
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
  int32_t n_qblocks;     // ceil(Q / kQueriesPerBlock)
  int32_t n_chunks;      // cloud splits of the full pass: chunk c covers points
  int32_t chunk_pts;     //   [c chunk_pts, min((c+1) chunk_pts, n_points))
  int64_t block_base;    // prefix of n_qblocks * n_chunks over sets
  // two-pass extension
  float* thresh;         // [n_qblocks] flag bound on the pass-A squared distance
  int32_t* list;         // [n_qblocks * qpbA] flagged queries, segment qb at qb * qpbA
                         //   (nullptr: exact set)
  int32_t* seg_count;    // [n_qblocks] flagged queries of each query block
  int2* work;            // [n_qblocks * n_tiles] (query block, tile << 4 | sub-tile mask):
                         //   some query of the block came under the bound in the tile
                         //   in pass A; bit j: sub-tile j's bounding box lies within
                         //   reach of the block's bounding box
  float4* fpos;          // [n_qblocks * qpbA] positions of the flagged queries, in the
                         //   order of `list` (written by the flag kernel)
  float* qbox;           // [ceil(n_points / kSubPts)][6] sub-tile bounding boxes (lo, hi)
  int64_t box_base;      // prefix of ceil(n_points / kSubPts) over two-pass sets
  int32_t* work_count;   // entries of `work` (zeroed by the rollout kernel)
  int64_t query_base;    // prefix of ceil(Q / kBlock) flag blocks over sets
  int32_t qpbA;          // positions per pass-A block (the variant's block size)
  int32_t n_tiles;       // ceil(n_points / kTilePts); pass-A chunks are whole tiles
  float d_max;
  const int32_t* perm;   // [Q] slot -> query, spatially sorted (nullptr: identity)
  unsigned* out_slot;    // two-pass sets: [Q] squared distances by slot (== out without
                         //   a sort); scattered back to `out` once pass B is done
  unsigned long long* nn;  // optional [n_qblocks * qpbA]: pass B also keeps
                           // (d^2 bits << 32 | index) per list slot (lowest index on ties)
  int32_t* nidx;           // with nn: [Q] nearest index per query (-1 where not flagged)
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

// Pass-A hit of query block qb (bounding box [blo, bhi]) in cloud tile `tile`:
// record the tile with the mask of its sub-tiles whose bounding box lies within
// squared distance r2 of the block's box.  With r2 = 2 thresh - d_max^2 (pass A errs by at most
// thresh - d_max^2, and a flagged query's pass-A value is below thresh) every point
// within d_max of a flagged query, and the point that flagged it, is in a recorded
// sub-tile; the relative margin covers the rounding of the box distance.
__device__ inline void append_hits(const QuerySet& S, int qb, int64_t tile, const float blo[3],
                                   const float bhi[3], float r2) {
  const float lim = r2 * (1.0f + 1e-5f) + 1e-6f;
  int mask = 0;
  for (int j = 0; j < kTileSplit; ++j) {
    const int64_t sub = tile * kTileSplit + j;
    if (sub * kSubPts >= S.n_points) break;
    const float* b = S.qbox + 6 * sub;
    float d2 = 0.0f;
    for (int a = 0; a < 3; ++a) {
      const float dd = fmaxf(0.0f, fmaxf(b[a] - bhi[a], blo[a] - b[3 + a]));
      d2 = fmaf(dd, dd, d2);
    }
    if (d2 <= lim) mask |= 1 << j;
  }
  if (mask) {
    const int e = atomicAdd(S.work_count, 1);
    S.work[e] = make_int2(qb, (int)(tile << 4) | mask);
  }
}

// Pass-A hit from a block whose per-wave query bounds are red[0..2][w] (min) and
// red[3..5][w] (max) in LDS.
__device__ inline void append_block_hits(const QuerySet& S, int qb, int64_t tile,
                                         const float (*red)[4], float r2) {
  float blo[3], bhi[3];
  for (int a = 0; a < 3; ++a) {
    blo[a] = fminf(fminf(red[a][0], red[a][1]), fminf(red[a][2], red[a][3]));
    bhi[a] = fmaxf(fmaxf(red[3 + a][0], red[3 + a][1]), fmaxf(red[3 + a][2], red[3 + a][3]));
  }
  append_hits(S, qb, tile, blo, bhi, r2);
}

// Squared reach of pass B around a block with pass-A bound thr (see append_hits).
__device__ inline float pass_b_reach2(float thr, float d_max) {
  return thr < INFINITY ? thr + (thr - d_max * d_max) : INFINITY;
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
                               hipStream_t s);
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
hipError_t launch_guides(const double p0[3], const double v0[3], const double a0[3],
                         const float* anchors, const float* end_vel, const float* end_acc,
                         double T, int M, float* coef, hipStream_t s);
hipError_t launch_rollout_noise(const DevProblem* d_probs, int n, int64_t total_samples,
                                int64_t total_elems, const DevParams& prm, const QuerySet* d_sets,
                                int64_t box_blocks, const void* h_blob, size_t blob_bytes,
                                hipStream_t s);
hipError_t launch_rollout(const DevProblem* d_probs, int n, int64_t total_samples,
                          const DevParams& prm, hipStream_t s);
hipError_t launch_min_dist(const QuerySet* d_sets, int n_sets, int64_t total_blocks,
                           hipStream_t s);
hipError_t launch_min_dist_approx(const QuerySet* d_sets, int n_sets, int64_t total_blocks,
                                  int variant, hipStream_t s);
hipError_t launch_min_dist_approx_matrix(const QuerySet* d_sets, int n_sets, int64_t total_blocks,
                                         int variant, hipStream_t s);
hipError_t launch_flag(const QuerySet* d_sets, int n_sets, int64_t total_queries, hipStream_t s);
hipError_t launch_min_dist_listed(const QuerySet* d_sets, int n_sets, int64_t total_blocks,
                                  hipStream_t s);
hipError_t launch_scatter_nearest(const QuerySet* d_sets, int n, hipStream_t s);
hipError_t launch_adjoint(const DevProblem* d_prob, const DevParams& prm, int64_t samples,
                          double* ckpt, double* seg, double* gsamp, hipStream_t s);
hipError_t launch_grad_reduce(const DevProblem* d_prob, const DevParams& prm, int64_t rows,
                              const double* gsamp, const float* grad_L, float* grad_u,
                              float* grad_w, double* wpart, hipStream_t s);
size_t grad_w_parts();  // doubles of the weight-gradient partial sums
hipError_t launch_finalize(const DevProblem* d_probs, int n, int64_t total_samples,
                           const DevParams& prm, bool write_s1, hipStream_t s);
hipError_t launch_update(const DevProblem* d_probs, int n, int64_t total_rows,
                         const DevParams& prm, hipStream_t s);
hipError_t launch_select_rollout(const DevSelect* d_sel, int n, int64_t total_inst,
                                 const DevParams& prm, const void* h_blob, size_t blob_bytes,
                                 hipStream_t s);
hipError_t launch_select_final(const DevSelect* d_sel, int n, const DevParams& prm,
                               hipStream_t s);

}  // namespace aero
