// C ABI entry points: host validation, workspace layout, descriptor staging and
// the launch sequence of each call.  See include/aero.h for the contract.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "aero_internal.h"

using namespace aero;

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
inline bool finite(float v) { return std::isfinite(v); }

// ---------------------------------------------------------------------------
// Descriptors reach the workspace through kernel arguments: the first kernel of a
// call carries them and writes them for the kernels that follow (or, when they do
// not fit in an argument, launch_put_bytes does), so every call enqueues kernels
// only: no host staging memory, no host-side synchronisation, and the calls can be
// captured into a graph by the caller.
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Optional per-kernel event timing.
// ---------------------------------------------------------------------------
struct Timing {
  bool on = false;
  struct Rec {
    int kernel;
    hipEvent_t a, b;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  double ms[AERO_K_COUNT] = {};
  int64_t n[AERO_K_COUNT] = {};
};
std::mutex g_tmu;
Timing g_timing;

hipEvent_t pool_event() {
  if (!g_timing.pool.empty()) {
    hipEvent_t e = g_timing.pool.back();
    g_timing.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

template <typename F>
hipError_t timed(int kernel, hipStream_t s, F&& launch) {
  if (!g_timing.on) return launch();
  std::lock_guard<std::mutex> lk(g_tmu);
  hipEvent_t a = pool_event(), b = pool_event();
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, s);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, s);
  g_timing.pending.push_back({kernel, a, b});
  return e;
}

// ---------------------------------------------------------------------------
// Online autotuner of the pass-A launch configuration (variant and persistent grid,
// kPassAConf), keyed by the call's shape.  The first kPassAConfigs calls of a shape
// time one configuration each with HIP events; the next reads them all and keeps the
// fastest.  Every configuration yields bitwise-identical costs and controls, so
// tuning never changes results.  While a stream is being captured into a graph no
// events are recorded and an unsettled shape uses the VALU pass.
// ---------------------------------------------------------------------------
struct TuneKey {
  int64_t q, p;
  int n;
  bool operator<(const TuneKey& o) const {
    return q != o.q ? q < o.q : p != o.p ? p < o.p : n < o.n;
  }
};
struct TuneState {
  int trials = 0;
  int choice = -1;
  hipEvent_t ev[kPassAConfigs][2] = {};
  float ms[kPassAConfigs] = {};
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneState> g_tune;
int g_forced_variant = -1;

TuneKey tune_key(const aero_problem* h, int n) {
  TuneKey k{0, 0, n};
  for (int b = 0; b < n; ++b) {
    k.q += (int64_t)h[b].M * h[b].N * h[b].K;
    k.p += h[b].n_points;
  }
  return k;
}

// The forced or already settled configuration of a shape, else the VALU pass (no
// trials).
int settled_config(const TuneKey& key) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (g_forced_variant >= 0) return g_forced_variant;
  auto it = g_tune.find(key);
  return (it != g_tune.end() && it->second.choice >= 0) ? it->second.choice : kPassAValu;
}

// Configuration for this call; *ev receives the event pair to record around pass A
// (or null).
int pick_config(const TuneKey& key, hipStream_t s, hipEvent_t** ev) {
  *ev = nullptr;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (g_forced_variant >= 0) return g_forced_variant;
  TuneState& st = g_tune[key];
  if (st.choice >= 0) return st.choice;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
    return kPassAValu;
  if (st.trials < kPassAConfigs) {
    const int v = st.trials;
    if (hipEventCreate(&st.ev[v][0]) != hipSuccess || hipEventCreate(&st.ev[v][1]) != hipSuccess)
      return kPassAValu;
    st.trials++;
    *ev = st.ev[v];
    return v;
  }
  // the trials are read without waiting: while the last one is still in flight this
  // call runs the VALU pass and a later call settles the shape
  for (int v = 0; v < kPassAConfigs; ++v)
    if (hipEventQuery(st.ev[v][1]) == hipErrorNotReady) return kPassAValu;
  int best = kPassAValu;
  for (int v = 0; v < kPassAConfigs; ++v) {
    if (hipEventElapsedTime(&st.ms[v], st.ev[v][0], st.ev[v][1]) != hipSuccess)
      st.ms[v] = 1e30f;
    hipEventDestroy(st.ev[v][0]);
    hipEventDestroy(st.ev[v][1]);
    if (st.ms[v] < st.ms[best]) best = v;
  }
  st.choice = best;
  return st.choice;
}

// ---------------------------------------------------------------------------
// Validation
// ---------------------------------------------------------------------------
int check_params(const aero_params* p) {
  if (!p) return AERO_ERR_NULL;
  const float* f = &p->dt;
  const size_t nf = offsetof(aero_params, seed) / sizeof(float);
  for (size_t i = 0; i < nf; ++i)
    if (!finite(f[i])) return AERO_ERR_PARAM;
  if (!(p->dt > 0.f) || !(p->lambda > 0.f) || !(p->mass > 0.f)) return AERO_ERR_PARAM;
  for (int c = 0; c < 4; ++c)
    if (p->sigma[c] < 0.f || p->u_min[c] > p->u_max[c]) return AERO_ERR_PARAM;
  if (p->C < 0.f || p->a < 0.f || p->d_min < 0.f || !(p->d_min < p->d_max)) return AERO_ERR_PARAM;
  if (p->reserved != 0) return AERO_ERR_PARAM;
  return AERO_OK;
}

int check_problem(const aero_problem& q, bool need_coef) {
  if (q.n_points < 0 || q.M < 1 || q.M > AERO_M_MAX || q.K < 1 || q.K > AERO_K_MAX || q.N < 2 ||
      q.N > AERO_N_MAX)
    return AERO_ERR_SHAPE;
  if ((q.n_points > 0 && !q.cloud) || !q.u_nom || (need_coef && !q.coef)) return AERO_ERR_NULL;
  for (float v : q.x0)
    if (!finite(v)) return AERO_ERR_PARAM;
  for (int i = 0; i < 3; ++i)
    if (!finite(q.p_goal[i]) || !finite(q.v_goal[i])) return AERO_ERR_PARAM;
  for (float v : q.q_goal)
    if (!finite(v)) return AERO_ERR_PARAM;
  const double qn = (double)q.x0[3] * q.x0[3] + (double)q.x0[4] * q.x0[4] +
                    (double)q.x0[5] * q.x0[5] + (double)q.x0[6] * q.x0[6];
  if (!(qn > 0.0)) return AERO_ERR_PARAM;
  return AERO_OK;
}

int check_problems(const aero_problem* h, int32_t n, bool need_coef) {
  if (!h) return AERO_ERR_NULL;
  if (n < 1 || n > AERO_BATCH_MAX) return AERO_ERR_SHAPE;
  int64_t total = 0;
  for (int b = 0; b < n; ++b) {
    const int e = check_problem(h[b], need_coef);
    if (e) return e;
    // positions are addressed by 32-bit slots (sort permutation, flag lists, nearest
    // indices): a problem, and the call, must stay below 2^31 of them
    const int64_t q = (int64_t)h[b].M * h[b].N * h[b].K;
    total += q;
    if (q >= AERO_POSITIONS_MAX || total >= AERO_POSITIONS_MAX) return AERO_ERR_SHAPE;
  }
  return AERO_OK;
}

DevParams promote(const aero_params& p) {
  DevParams d;
  d.dt = p.dt;
  d.lambda = p.lambda;
  d.mass = p.mass;
  d.gravity = p.gravity;
  for (int c = 0; c < 4; ++c) {
    d.sigma[c] = p.sigma[c];
    d.u_min[c] = p.u_min[c];
    d.u_max[c] = p.u_max[c];
  }
  d.Q_track = p.Q_track;
  d.Q_vnorm = p.Q_vnorm;
  d.Q_c = p.Q_c;
  d.Q_cdelta = p.Q_cdelta;
  d.Q_p = p.Q_p;
  d.Q_v = p.Q_v;
  d.Q_q = p.Q_q;
  d.C = p.C;
  d.a = p.a;
  d.d_min = p.d_min;
  d.d_max = p.d_max;
  for (int i = 0; i < 5; ++i) d.w[i] = p.w[i];
  d.seed_lo = (uint32_t)(p.seed & 0xFFFFFFFFu);
  d.seed_hi = (uint32_t)(p.seed >> 32);
  d.iter_base = p.iter_base;
  d.pad = 0;
  return d;
}

// ---------------------------------------------------------------------------
// Workspace layout
// ---------------------------------------------------------------------------
struct Cursor {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off = align_up(off + count * sizeof(T));
    return p;
  }
};

// Fewest cloud tiles, and fewest positions, for which the positions (and the cloud)
// are spatially sorted before the cull step.  A few thousand positions make a few
// query blocks: sorting the whole cloud for them costs more than it saves.
constexpr int kSortMinTiles = 16;
constexpr int64_t kSortMinQueries = 8192;

bool sorts(const aero_problem& q) {
  return q.n_points > 0 && ((int64_t)q.n_points + kTilePts - 1) / kTilePts >= kSortMinTiles &&
         (int64_t)q.M * q.N * q.K >= kSortMinQueries;
}

// Split P points into about `want` chunks of a multiple of `align` points (exact sets).
void set_chunks(int64_t P, int64_t want, int32_t& n_chunks, int32_t& chunk_pts,
                int64_t align = 64) {
  if (P <= 0) {
    n_chunks = 0;
    chunk_pts = 0;
    return;
  }
  want = std::min<int64_t>(std::max<int64_t>(want, 1), (P + align - 1) / align);
  const int64_t per = (P + want - 1) / want;
  chunk_pts = (int32_t)((per + align - 1) / align * align);
  n_chunks = (int32_t)((P + chunk_pts - 1) / chunk_pts);
}

// Whether the cull step limits each query block to the sub-tiles within its reach
// (0: every sub-tile is listed, which turns the two passes back into brute force).
int g_cull = 1;

struct MppiPlan {
  std::vector<DevProblem> probs;
  std::vector<QuerySet> sets;
  std::vector<SortSet> sorts;   // two per problem: positions, then the cloud
  DevProblem* d_probs = nullptr;
  QuerySet* d_sets = nullptr;
  SortSet* d_sorts = nullptr;   // adjacent to d_sets: one descriptor upload
  int64_t total_samples = 0, total_rows = 0, total_inst = 0;
  int64_t sort_blocks = 0;
  int sort_per_thread = 1;      // elements per thread of the sort's tiles
  int64_t total_tiles = 0;      // cloud tiles of the two-pass sets (box launches)
  int64_t total_qblocks = 0;    // query blocks of the two-pass sets (cull launch)
  int64_t item_cap = 0;         // capacity of the call's item list
  int64_t total_elems = 0;      // sum of M*N*K (rollout noise draws)
  int2* items = nullptr;
  int32_t* item_count = nullptr;
  unsigned char* hitf = nullptr;
  uint32_t* hmask = nullptr;    // the call's hit words (see QuerySet::hmask)
  int64_t mask_words = 0;
  bool any_sorted = false;      // some set works in sorted slots
  bool any_scloud = false;      // some set has a sorted cloud
  bool any_nn = false;          // some set records nearest indices
  size_t bytes = 0;
};

void plan_mppi(const aero_problem* h, int n, char* ws, float d_max, MppiPlan& pl,
               int variant = kPassAValu, bool track_nearest = false) {
  Cursor cur{ws};
  pl.d_probs = cur.take<DevProblem>(n);
  pl.d_sets = cur.take<QuerySet>(n);
  pl.d_sorts = cur.take<SortSet>(2 * n);
  pl.probs.assign(n, DevProblem{});
  pl.sets.assign(n, QuerySet{});
  pl.sorts.assign(2 * n, SortSet{});
  const int qpbA = kPassAQPB[variant];
  // the call's item list: a block lists each sub-tile at most once, so the blocks of
  // the smallest block size times the sub-tiles bound it (the layout does not depend
  // on the variant)
  int64_t cap = 0;
  for (int b = 0; b < n; ++b)
    if (h[b].n_points > 0) {
      const int64_t Q = (int64_t)h[b].M * h[b].N * h[b].K;
      cap += (Q + kPassAMinQPB - 1) / kPassAMinQPB * (((int64_t)h[b].n_points + kSubPts - 1) / kSubPts);
    }
  pl.item_cap = cap;
  pl.items = cur.take<int2>(cap);
  pl.hitf = cur.take<unsigned char>(cap);
  pl.item_count = cur.take<int32_t>(1);
  // hit words: item i's at i * qpbA / 32.  A call whose every listable item had its
  // words would need cap * 16 words (cap counts 512-position blocks); this holds an
  // eighth of that, and at least 4 MiB: items past it are taken whole by pass B
  // (every query of the block), which is exact, only slower.
  pl.mask_words = cap > 0 ? std::max<int64_t>(int64_t(1) << 20, 2 * cap) : 0;
  pl.hmask = cur.take<uint32_t>(pl.mask_words);
  int64_t sort_blocks = 0, eb = 0, sb = 0, rb = 0, qbb = 0, tb = 0, ib = 0;
  // the sort's tile: as many elements per thread as still leave about kSortMinGrid
  // tiles over the call's sorted positions and clouds
  int64_t sort_elems = 0;
  for (int b = 0; b < n; ++b)
    if (sorts(h[b]))
      sort_elems += (int64_t)h[b].M * h[b].N * h[b].K + h[b].n_points;
  int spt = 1;
  while (spt < kSortMaxPerThread && sort_elems / (2 * spt * kBlock) >= kSortMinGrid) spt *= 2;
  pl.sort_per_thread = spt;
  const int64_t sort_tile = (int64_t)spt * kBlock;
  for (int b = 0; b < n; ++b) {
    const aero_problem& q = h[b];
    DevProblem& d = pl.probs[b];
    const int64_t MK = (int64_t)q.M * q.K, MN = (int64_t)q.M * q.N, MNK = MN * q.K;
    d.cloud = q.cloud;
    d.n_points = q.n_points;
    d.M = q.M;
    d.K = q.K;
    d.N = q.N;
    d.problem_id = q.problem_id;
    memcpy(d.x0, q.x0, sizeof d.x0);
    memcpy(d.pg, q.p_goal, sizeof d.pg);
    memcpy(d.vg, q.v_goal, sizeof d.vg);
    memcpy(d.qg, q.q_goal, sizeof d.qg);
    d.coef = q.coef;
    d.u_nom = q.u_nom;
    d.w_dev = q.w;
    d.J_ctrl = cur.take<double>(MK);
    double* s1 = cur.take<double>(q.S1 ? 0 : MK);
    d.S1 = q.S1 ? q.S1 : s1;
    float* de = cur.take<float>(q.delta_eff ? 0 : MNK * 4);
    d.deff = q.delta_eff ? q.delta_eff : de;
    d.pos = cur.take<float>(3 * MNK);
    unsigned* md = cur.take<unsigned>(q.min_dist2 ? 0 : MNK);
    d.mind2 = q.min_dist2 ? reinterpret_cast<unsigned*>(q.min_dist2) : md;
    d.sample_base = sb;
    d.row_base = rb;
    d.inst_base = ib;
    d.wexp = cur.take<double>(MK);
    d.eta = cur.take<double>(q.M);
    ib += q.M;
    d.elem_base = eb;
    d.noise = cur.take<double>(4 * MNK);
    d.state = cur.take<float>(10 * MNK);
    d.item_count = pl.item_count;
    sb += MK;
    rb += MN;
    eb += MNK;

    QuerySet& qs = pl.sets[b];
    qs.px = d.pos;
    qs.py = d.pos ? d.pos + MNK : nullptr;
    qs.pz = d.pos ? d.pos + 2 * MNK : nullptr;
    qs.sp = d.pos;  // planes at stride Q; the spatial sort replaces it below
    qs.out = d.mind2;
    qs.cloud = q.cloud;
    qs.Q = MNK;
    qs.n_points = q.n_points;
    qs.qpbA = qpbA;
    qs.d_max = d_max;
    qs.cull = g_cull;
    const bool two_pass = q.n_points > 0;
    const int64_t n_tiles = ((int64_t)q.n_points + kTilePts - 1) / kTilePts;
    const int64_t n_sub = ((int64_t)q.n_points + kSubPts - 1) / kSubPts;
    qs.n_qblocks = two_pass ? (int)((MNK + qpbA - 1) / qpbA) : 0;
    qs.n_tiles = (int32_t)n_tiles;
    qs.qb_base = qbb;
    qs.tile_base = tb;
    if (two_pass) {
      qbb += qs.n_qblocks;
      tb += n_tiles;
      // sized for the smallest block size (the most blocks), so the layout does not
      // depend on the variant
      const int64_t max_blocks = (MNK + kPassAMinQPB - 1) / kPassAMinQPB;
      qs.binfo = cur.take<float4>(max_blocks);
      qs.tbox = cur.take<float>(6 * n_tiles);
      qs.sbox = cur.take<float>(6 * n_sub);
      qs.gbox = cur.take<float>(6 * n_sub * kGroupsPerSub);
      qs.ubox = cur.take<float>(6 * ((n_tiles + kSuperTiles - 1) / kSuperTiles));
      qs.amin = cur.take<unsigned>(MNK);  // reset by the noise kernel
      d.amin = qs.amin;
      qs.items = pl.items;
      qs.item_count = pl.item_count;
      qs.hitf = pl.hitf;
      qs.hmask = pl.hmask;
      qs.mask_words = pl.mask_words;
    }
    // spatial order of the positions, and of the cloud, for the cull step
    SortSet& so = pl.sorts[2 * b];
    SortSet& sc = pl.sorts[2 * b + 1];
    so.block_base = sort_blocks;
    if (two_pass && sorts(q)) {
      so.px = qs.px;
      so.py = qs.py;
      so.pz = qs.pz;
      so.stride = 1;
      so.Q = MNK;
      so.n_blocks = (int32_t)((MNK + sort_tile - 1) / sort_tile);
      so.box = cur.take<unsigned>(kBoxCopies * kBoxStride);
      so.key[0] = cur.take<uint32_t>(MNK);
      so.key[1] = cur.take<uint32_t>(MNK);
      so.val[0] = cur.take<int32_t>(MNK);
      so.val[1] = cur.take<int32_t>(MNK);
      so.inv = cur.take<int32_t>(MNK);
      so.sp = cur.take<float>(3 * MNK);
      so.tp = cur.take<float>(3 * MNK);
      so.table = cur.take<int32_t>((int64_t)kSortDigits * so.n_blocks);
      so.rowsum = cur.take<int32_t>(kSortDigits);
      sort_blocks += so.n_blocks;
      qs.perm = so.val[kSortPasses % 2];  // where the last pass leaves it
      qs.sp = so.sp;
      qs.out_slot = cur.take<unsigned>(MNK);
      d.sort_box = so.box;
      d.out_slot = qs.out_slot;
      d.inv = so.inv;
      pl.any_sorted = true;
      // the cloud, keyed on the positions' box widened by d_max and a metre
      const int64_t P = q.n_points;
      sc.block_base = sort_blocks;
      sc.px = q.cloud;
      sc.py = q.cloud ? q.cloud + 1 : nullptr;
      sc.pz = q.cloud ? q.cloud + 2 : nullptr;
      sc.stride = 3;
      sc.Q = P;
      sc.n_blocks = (int32_t)((P + sort_tile - 1) / sort_tile);
      sc.box = so.box;
      sc.margin = d_max + 1.0f;
      sc.key[0] = cur.take<uint32_t>(P);
      sc.key[1] = cur.take<uint32_t>(P);
      sc.val[0] = cur.take<int32_t>(P);
      sc.val[1] = cur.take<int32_t>(P);
      sc.table = cur.take<int32_t>((int64_t)kSortDigits * sc.n_blocks);
      sc.rowsum = cur.take<int32_t>(kSortDigits);
      sc.sc = cur.take<float4>(P);
      sc.tp = cur.take<float>(3 * P);
      sort_blocks += sc.n_blocks;
      qs.scloud = sc.sc;
      qs.stbox = cur.take<float>(6 * n_tiles);
      qs.ssbox = cur.take<float>(6 * n_sub);
      qs.sgbox = cur.take<float>(6 * n_sub * kGroupsPerSub);
      qs.subox = cur.take<float>(6 * ((n_tiles + kSuperTiles - 1) / kSuperTiles));
      pl.any_scloud = true;
    } else {
      sc.block_base = sort_blocks;
    }
    if (!qs.out_slot) qs.out_slot = qs.out;
    // nearest indices requested by the caller of a forward step
    if (track_nearest && q.nearest_idx) {
      d.nidx = q.nearest_idx;  // reset to -1 by the noise kernel
      if (two_pass) {
        qs.nn = cur.take<unsigned long long>(MNK);  // reset by the noise kernel
        qs.nidx = q.nearest_idx;
        d.nn = qs.nn;
        pl.any_nn = true;
      }
    }
  }
  pl.total_samples = sb;
  pl.total_rows = rb;
  pl.total_inst = ib;
  pl.total_tiles = tb;
  pl.total_qblocks = qbb;
  pl.sort_blocks = sort_blocks;
  pl.total_elems = eb;
  pl.bytes = cur.off;
}

// The image of a plan's problem, query-set and sort descriptors (adjacent in the
// workspace from d_probs on), written to the workspace by the noise launch.
std::vector<char> mppi_blob(const MppiPlan& pl, int n) {
  const char* b0 = (const char*)pl.d_probs;
  std::vector<char> blob((const char*)pl.d_sorts - b0 + 2 * n * sizeof(SortSet));
  memcpy(blob.data(), pl.probs.data(), n * sizeof(DevProblem));
  memcpy(blob.data() + ((const char*)pl.d_sets - b0), pl.sets.data(), n * sizeof(QuerySet));
  memcpy(blob.data() + ((const char*)pl.d_sorts - b0), pl.sorts.data(), 2 * n * sizeof(SortSet));
  return blob;
}

// The distance passes of a planned Stage-I call: the spatial sorts, the cull step,
// pass A (timed by `tev` when given) and pass B.
hipError_t run_distance(const MppiPlan& pl, int n, int cfg, hipEvent_t* tev, hipStream_t s) {
  hipError_t he = hipSuccess;
  const int variant = kPassAConf[cfg].variant;
  if (pl.sort_blocks > 0)
    he = timed(AERO_K_SORT, s,
               [&] {
                 return launch_spatial_sort(pl.d_sorts, 2 * n, pl.sort_blocks, pl.sort_per_thread,
                                            s);
               });
  if (he == hipSuccess && pl.total_qblocks > 0)
    he = timed(AERO_K_CULL, s, [&] {
      hipError_t e = pl.any_scloud ? launch_sorted_boxes(pl.d_sets, n, pl.total_tiles, s)
                                   : hipSuccess;
      return e == hipSuccess ? launch_cull(pl.d_sets, n, pl.total_qblocks, variant, s) : e;
    });
  if (he == hipSuccess && tev) he = hipEventRecord(tev[0], s);
  if (he == hipSuccess && pl.item_cap > 0)
    he = timed(AERO_K_MIN_DIST, s, [&] {
      return launch_pass_a(pl.d_sets, n, pl.items, pl.item_count, pl.hitf, pl.item_cap, variant,
                           kPassAConf[cfg].grid, s);
    });
  if (he == hipSuccess && tev) he = hipEventRecord(tev[1], s);
  if (he == hipSuccess && pl.item_cap > 0)
    he = timed(AERO_K_MIN_DIST_EXACT, s, [&] {
      return launch_pass_b(pl.d_sets, n, pl.items, pl.item_count, pl.hitf, pl.item_cap,
                           pl.any_nn, s);
    });
  return he;
}

struct BackwardPlan {
  MppiPlan fwd;
  double* J = nullptr;
  int32_t* nidx = nullptr;
  unsigned long long* nn = nullptr;
  double* ckpt = nullptr;
  double* seg = nullptr;
  double* gsamp = nullptr;
  double* wpart = nullptr;
  size_t bytes = 0;
};

void plan_backward(const aero_problem* h, char* ws, float d_max, BackwardPlan& bp,
                   int variant = kPassAValu) {
  plan_mppi(h, 1, ws, d_max, bp.fwd, variant);
  Cursor cur{ws};
  cur.off = bp.fwd.bytes;
  const aero_problem& q = h[0];
  const int64_t MK = (int64_t)q.M * q.K, MNK = MK * q.N;
  const int64_t n_seg = (q.N + 7) / 8;
  bp.J = cur.take<double>(5 * MK);
  int32_t* ni = cur.take<int32_t>(q.nearest_idx ? 0 : MNK);
  bp.nidx = q.nearest_idx ? q.nearest_idx : ni;
  bp.nn = cur.take<unsigned long long>(q.n_points > 0 ? MNK : 0);
  bp.ckpt = cur.take<double>(n_seg * 10 * MK);
  bp.seg = cur.take<double>(8 * 10 * MK);
  bp.gsamp = cur.take<double>(MNK * 4);
  bp.wpart = cur.take<double>(grad_w_parts());
  bp.bytes = cur.off;
  if (ws) {
    DevProblem& d = bp.fwd.probs[0];
    d.J = bp.J;
    d.nidx = bp.nidx;
    QuerySet& qs = bp.fwd.sets[0];
    if (q.n_points > 0) {
      qs.nn = bp.nn;
      qs.nidx = bp.nidx;
      d.nn = bp.nn;  // reset by the noise kernel
      bp.fwd.any_nn = true;
    }
  }
}

// Host records of a Stage-II call live in arrays that the caller of plan_select
// provides (heap vectors for the workspace entry point, stack arrays for the one that
// allocates nothing).
struct SelectPlan {
  DevSelect* sel = nullptr;     // [n] host records
  QuerySet* sets = nullptr;     // [n]
  DevSelect* d_sel = nullptr;
  QuerySet* d_sets = nullptr;
  int64_t total_inst = 0, total_blocks = 0;
  size_t bytes = 0;
};

// Queries per block of an exact set: kBlock lanes times 1, 2, 4 or 8 queries each,
// the fewest that keep the set within kExactQueryBlocks blocks.  Few queries per lane
// keep each wave's queries (consecutive positions of one or two rollouts) in a small
// box, so that the wave skips most cloud tiles; more blocks read the cloud more often.
constexpr int64_t kExactQueryBlocks = 16;
int64_t exact_block_queries(int64_t Q) {
  int64_t r = 1;
  while (r < kQueriesPerLane && r * kBlock * kExactQueryBlocks < Q) r *= 2;
  return r * kBlock;
}

void plan_select(const aero_problem* h, int n, char* ws, double* S2, int32_t* best,
                 SelectPlan& pl) {
  Cursor cur{ws};
  pl.d_sel = cur.take<DevSelect>(n);
  pl.d_sets = cur.take<QuerySet>(n);
  for (int b = 0; b < n; ++b) {
    pl.sel[b] = DevSelect{};
    pl.sets[b] = QuerySet{};
  }
  int64_t qblocks = 0;
  for (int b = 0; b < n; ++b)
    if (h[b].n_points > 0) {
      const int64_t qpb = exact_block_queries((int64_t)h[b].M * h[b].N);
      qblocks += ((int64_t)h[b].M * h[b].N + qpb - 1) / qpb;
    }
  int64_t ib = 0, blk = 0;
  for (int b = 0; b < n; ++b) {
    const aero_problem& q = h[b];
    DevSelect& d = pl.sel[b];
    const int64_t MN = (int64_t)q.M * q.N;
    d.cloud = q.cloud;
    d.n_points = q.n_points;
    d.M = q.M;
    d.N = q.N;
    memcpy(d.x0, q.x0, sizeof d.x0);
    memcpy(d.pg, q.p_goal, sizeof d.pg);
    memcpy(d.vg, q.v_goal, sizeof d.vg);
    memcpy(d.qg, q.q_goal, sizeof d.qg);
    d.u_nom = q.u_nom;
    d.w_dev = q.w;
    d.state = cur.take<double>(10 * MN);
    d.pos = cur.take<float>(3 * MN);
    d.mind2 = cur.take<unsigned>(kSelCopies * MN);
    d.S2 = S2 ? S2 + ib : nullptr;
    d.best = best ? best + b : nullptr;
    d.inst_base = ib;
    ib += q.M;
    QuerySet& qs = pl.sets[b];
    qs.px = d.pos;
    qs.py = d.pos ? d.pos + MN : nullptr;
    qs.pz = d.pos ? d.pos + 2 * MN : nullptr;
    qs.sp = d.pos;
    qs.out = d.mind2;
    qs.n_copies = kSelCopies;  // hundreds of workgroups meet on each query's minimum
    qs.cloud = q.cloud;
    qs.Q = MN;
    qs.n_points = q.n_points;
    qs.qpbA = (int32_t)exact_block_queries(MN);
    qs.n_qblocks = (int)((MN + qs.qpbA - 1) / qs.qpbA);
    // few queries: split the cloud so that about 512 workgroups share the work (the
    // pass is latency-bound at this size), with at most one tile of points each (the
    // work of a chunk is concentrated in the tiles near the rollouts)
    set_chunks(q.n_points,
               std::max<int64_t>((512 + qblocks - 1) / std::max<int64_t>(qblocks, 1),
                                 (q.n_points + kTilePts - 1) / kTilePts),
               qs.n_chunks, qs.chunk_pts);
    qs.block_base = blk;
    blk += (int64_t)qs.n_qblocks * qs.n_chunks;
  }
  (void)qblocks;
  pl.total_inst = ib;
  pl.total_blocks = blk;
  pl.bytes = cur.off;
}

inline int dev_status(hipError_t e) { return e == hipSuccess ? AERO_OK : AERO_ERR_DEVICE; }

// A launch bracketed by the optional event timers, or plain (the entry point that
// allocates nothing records no events: creating one may allocate).
template <typename F>
hipError_t maybe_timed(bool timing, int kernel, hipStream_t s, F&& launch) {
  return timing ? timed(kernel, s, launch) : launch();
}

// Descriptor image of a Stage-II plan (records then query sets, at their workspace
// offsets) in `blob`, which holds select_blob_bytes(pl, n) bytes; returns that size.
size_t select_blob_bytes(const SelectPlan& pl, int n) {
  return (size_t)((const char*)pl.d_sets - (const char*)pl.d_sel) + n * sizeof(QuerySet);
}
size_t select_blob(const SelectPlan& pl, int n, char* blob) {
  const size_t off = (const char*)pl.d_sets - (const char*)pl.d_sel;
  memset(blob, 0, off);
  memcpy(blob, pl.sel, n * sizeof(DevSelect));
  memcpy(blob + off, pl.sets, n * sizeof(QuerySet));
  return off + n * sizeof(QuerySet);
}

// The launch sequence of a planned Stage-II call (the plan is laid out in its workspace).
hipError_t run_select(const SelectPlan& pl, int n, const DevParams& prm, const char* blob,
                      size_t blob_bytes, bool timing, hipStream_t s) {
  hipError_t he = maybe_timed(timing, AERO_K_SEL_ROLLOUT, s, [&] {
    return launch_select_rollout(pl.d_sel, n, pl.total_inst, prm, blob, blob_bytes, s);
  });
  if (he == hipSuccess && pl.total_blocks > 0)
    he = maybe_timed(timing, AERO_K_SEL_MIN_DIST, s,
                     [&] { return launch_min_dist(pl.d_sets, n, pl.total_blocks, (float)prm.d_max, s); });
  if (he == hipSuccess)
    he = maybe_timed(timing, AERO_K_SEL_FINAL, s,
                     [&] { return launch_select_final(pl.d_sel, n, prm, s); });
  return he;
}

// ---------------------------------------------------------------------------
// Workspace of aero_select_best_noalloc: a file-scope device array, of which every
// GPU holds its own copy (at its own address) from the first call on it until the
// process ends.  Host code never names the array in a launch or copy: it uses the
// address that hipGetSymbolAddress returned on that device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[AERO_NOALLOC_SCRATCH_BYTES];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};

// The current device's copy of `scratch`, looked up once per device with that device
// current; nullptr if the runtime reports an error.
void* scratch_address() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// Stack room for the descriptor image of AERO_NOALLOC_BATCH_MAX problems.
constexpr size_t kNoAllocBlobBytes =
    (AERO_NOALLOC_BATCH_MAX * sizeof(DevSelect) + kAlign - 1) / kAlign * kAlign +
    AERO_NOALLOC_BATCH_MAX * sizeof(QuerySet);

void table_angles(int32_t n_az, int32_t n_el, float* out) {
  float* az_b = out;
  float* el_b = az_b + 2 * n_az;
  float* az_c = el_b + 2 * (n_el + 1);
  float* el_c = az_c + 2 * n_az;
  for (int i = 0; i < n_az; ++i) {
    const double t = -M_PI + 2.0 * M_PI * (double)i / (double)n_az;
    az_b[2 * i] = (float)cos(t);
    az_b[2 * i + 1] = (float)sin(t);
    const double tc = -M_PI + 2.0 * M_PI * ((double)i + 0.5) / (double)n_az;
    az_c[2 * i] = (float)cos(tc);
    az_c[2 * i + 1] = (float)sin(tc);
  }
  for (int j = 0; j <= n_el; ++j) {
    const double t = -0.5 * M_PI + M_PI * (double)j / (double)n_el;
    el_b[2 * j] = (float)cos(t);
    el_b[2 * j + 1] = (float)sin(t);
  }
  for (int j = 0; j < n_el; ++j) {
    const double t = -0.5 * M_PI + M_PI * ((double)j + 0.5) / (double)n_el;
    el_c[2 * j] = (float)cos(t);
    el_c[2 * j + 1] = (float)sin(t);
  }
}

}  // namespace

extern "C" {

const char* aero_status_string(int status) {
  switch (status) {
    case AERO_OK: return "AERO_OK: success";
    case AERO_ERR_NULL: return "AERO_ERR_NULL: a required pointer is NULL";
    case AERO_ERR_SHAPE: return "AERO_ERR_SHAPE: a size is out of range";
    case AERO_ERR_PARAM: return "AERO_ERR_PARAM: a parameter is non-finite or out of its domain";
    case AERO_ERR_WORKSPACE: return "AERO_ERR_WORKSPACE: workspace missing or too small";
    case AERO_ERR_DEVICE: return "AERO_ERR_DEVICE: the HIP runtime reported an error";
    default: return "unknown aero_status";
  }
}

size_t aero_partition_tables_size(int32_t n_az, int32_t n_el) {
  if (n_az < 1 || n_el < 1) return 0;
  return (size_t)2 * n_az + 2 * (n_el + 1) + 2 * n_az + 2 * n_el;
}

int aero_partition_tables(int32_t n_az, int32_t n_el, float* h_out, size_t n_floats) {
  if (!h_out) return AERO_ERR_NULL;
  if (n_az < 3 || n_el < 1 || n_az > AERO_GRID_MAX || n_el > AERO_GRID_MAX) return AERO_ERR_SHAPE;
  if (n_floats < aero_partition_tables_size(n_az, n_el)) return AERO_ERR_SHAPE;
  table_angles(n_az, n_el, h_out);
  return AERO_OK;
}

size_t aero_workspace_size(int which, const aero_problem* h, int32_t n) {
  if (!h || n < 1 || n > AERO_BATCH_MAX) return 0;
  for (int b = 0; b < n; ++b)
    if (h[b].M < 1 || h[b].K < 1 || h[b].N < 2 || h[b].n_points < 0) return 0;
  if (which == AERO_CALL_MPPI_STEP) {
    MppiPlan pl;
    plan_mppi(h, n, nullptr, 1.0f, pl, kPassAValu, true);
    return pl.bytes;
  }
  if (which == AERO_CALL_BACKWARD) {
    if (n != 1) return 0;
    BackwardPlan bp;
    plan_backward(h, nullptr, 1.0f, bp);
    return bp.bytes;
  }
  if (which == AERO_CALL_SELECT_BEST) {
    std::vector<DevSelect> sel(n);
    std::vector<QuerySet> sets(n);
    SelectPlan pl;
    pl.sel = sel.data();
    pl.sets = sets.data();
    plan_select(h, n, nullptr, nullptr, nullptr, pl);
    return pl.bytes;
  }
  return 0;
}

namespace {

// Host checks of aero_partition_anchors (outputs and tables present, grid and block in
// range, finite parameters).
int check_partition(const aero_partition_spec* spec, const float* d_cloud, int32_t n_points,
                    const float* goal_dir, const void* d_fine_key, const void* d_fine_idx,
                    const void* d_coarse_best, const void* d_anchor_cell,
                    const void* d_anchor_fine, const void* d_anchors) {
  if (!spec || !goal_dir || !d_fine_key || !d_fine_idx || !d_coarse_best || !d_anchor_cell ||
      !d_anchor_fine || !d_anchors || !spec->d_tables)
    return AERO_ERR_NULL;
  if (n_points < 0) return AERO_ERR_SHAPE;
  if (n_points > 0 && !d_cloud) return AERO_ERR_NULL;
  if (spec->n_az_c < 1 || spec->n_el_c < 1 || spec->f_a < 1 || spec->f_e < 1)
    return AERO_ERR_SHAPE;
  const int64_t n_az = (int64_t)spec->n_az_c * spec->f_a, n_el = (int64_t)spec->n_el_c * spec->f_e;
  if (n_az < 3 || n_az > AERO_GRID_MAX || n_el > AERO_GRID_MAX) return AERO_ERR_SHAPE;
  if (spec->M_h < 1 || spec->M_h > spec->n_az_c || spec->M_v < 1 || spec->M_v > spec->n_el_c ||
      spec->M_h * spec->M_v > AERO_M_MAX)
    return AERO_ERR_SHAPE;
  if (!finite(spec->r_max) || !(spec->r_max > 0.f) || !finite(spec->ell)) return AERO_ERR_PARAM;
  for (int i = 0; i < 3; ++i)
    if (!finite(spec->p0[i]) || !finite(goal_dir[i])) return AERO_ERR_PARAM;
  return AERO_OK;
}

}  // namespace

int aero_partition_anchors(const aero_partition_spec* spec, const float* d_cloud, int32_t n_points,
                           const float* h_goal_dir, double* d_fine_key, int32_t* d_fine_idx,
                           int32_t* d_coarse_best, int32_t* d_anchor_cell, int32_t* d_anchor_fine,
                           float* d_anchors, void* stream) {
  const int e = check_partition(spec, d_cloud, n_points, h_goal_dir, d_fine_key, d_fine_idx,
                                d_coarse_best, d_anchor_cell, d_anchor_fine, d_anchors);
  if (e) return e;
  const hipStream_t s = (hipStream_t)stream;
  return dev_status(timed(AERO_K_PARTITION, s, [&] {
    return launch_partition(*spec, d_cloud, n_points, h_goal_dir, d_fine_key, d_fine_idx,
                            d_coarse_best, d_anchor_cell, d_anchor_fine, d_anchors, s);
  }));
}


size_t aero_front_end_workspace_size(int32_t n) {
  if (n < 1 || n > AERO_BATCH_MAX) return 0;
  return align_up((size_t)n * sizeof(FrontJob));
}

int aero_front_end(const aero_front_end_job* h, int32_t n, void* d_ws, size_t ws_bytes,
                   void* stream) {
  if (!h) return AERO_ERR_NULL;
  if (n < 1 || n > AERO_BATCH_MAX) return AERO_ERR_SHAPE;
  std::vector<FrontJob> jobs(n);
  int64_t cells = 0, blocks = 0;
  for (int b = 0; b < n; ++b) {
    const aero_front_end_job& q = h[b];
    const int e = check_partition(&q.spec, q.d_cloud, q.n_points, q.goal_dir, q.d_fine_key,
                                  q.d_fine_idx, q.d_coarse_best, q.d_anchor_cell, q.d_anchor_fine,
                                  q.d_anchors);
    if (e) return e;
    if (!q.d_coef) return AERO_ERR_NULL;
    if (!finite(q.horizon_T) || !(q.horizon_T > 0.f)) return AERO_ERR_PARAM;
    for (int i = 0; i < 3; ++i)
      if (!finite(q.v0[i]) || !finite(q.a0[i])) return AERO_ERR_PARAM;
    FrontJob& J = jobs[b];
    J.tables = q.spec.d_tables;
    J.cloud = q.n_points > 0 ? q.d_cloud : nullptr;
    J.key = reinterpret_cast<unsigned long long*>(q.d_fine_key);
    J.idx = reinterpret_cast<unsigned*>(q.d_fine_idx);
    J.coarse_best = q.d_coarse_best;
    J.anchor_cell = q.d_anchor_cell;
    J.anchor_fine = q.d_anchor_fine;
    J.anchors = q.d_anchors;
    J.coef = q.d_coef;
    J.end_vel = q.d_end_vel;
    J.end_acc = q.d_end_acc;
    J.cell_base = cells;
    J.block_base = blocks;
    J.n_points = q.n_points;
    J.n_az_c = q.spec.n_az_c;
    J.n_el_c = q.spec.n_el_c;
    J.f_a = q.spec.f_a;
    J.f_e = q.spec.f_e;
    J.M_h = q.spec.M_h;
    J.M_v = q.spec.M_v;
    J.pad = 0;
    J.r_max = q.spec.r_max;
    J.ell = q.spec.ell;
    J.T = q.horizon_T;
    J.pad1 = 0.f;
    for (int i = 0; i < 3; ++i) {
      J.p0[i] = q.spec.p0[i];
      J.goal[i] = q.goal_dir[i];
      J.v0[i] = q.v0[i];
      J.a0[i] = q.a0[i];
    }
    cells += (int64_t)q.spec.n_az_c * q.spec.f_a * q.spec.n_el_c * q.spec.f_e;
    blocks += (q.n_points + kBlock - 1) / kBlock;
  }
  if (!d_ws || ws_bytes < aero_front_end_workspace_size(n)) return AERO_ERR_WORKSPACE;
  const hipStream_t s = (hipStream_t)stream;
  return dev_status(timed(AERO_K_PARTITION, s, [&] {
    return launch_front_end(static_cast<FrontJob*>(d_ws), jobs.data(), n, cells, blocks, s);
  }));
}

int aero_filtered_cloud(const float* d_cloud, int32_t n_points, const int32_t* d_fine_idx,
                        int32_t n_fine, float* d_out, void* stream) {
  if (!d_fine_idx || !d_out) return AERO_ERR_NULL;
  if (n_points < 0 || n_fine < 1) return AERO_ERR_SHAPE;
  if (n_points > 0 && !d_cloud) return AERO_ERR_NULL;
  const hipStream_t s = (hipStream_t)stream;
  return dev_status(timed(AERO_K_PARTITION, s, [&] {
    return launch_filter_cloud(d_cloud, n_points, d_fine_idx, n_fine, d_out, s);
  }));
}

int aero_build_guides(const float* h_p0, const float* h_v0, const float* h_a0,
                      const float* d_anchors, const float* d_end_vel, const float* d_end_acc,
                      float horizon_T, int32_t M, float* d_coef, void* stream) {
  if (!h_p0 || !h_v0 || !h_a0 || !d_anchors || !d_coef) return AERO_ERR_NULL;
  if (M < 1 || M > AERO_M_MAX) return AERO_ERR_SHAPE;
  if (!finite(horizon_T) || !(horizon_T > 0.f)) return AERO_ERR_PARAM;
  double p0[3], v0[3], a0[3];
  for (int i = 0; i < 3; ++i) {
    if (!finite(h_p0[i]) || !finite(h_v0[i]) || !finite(h_a0[i])) return AERO_ERR_PARAM;
    p0[i] = h_p0[i];
    v0[i] = h_v0[i];
    a0[i] = h_a0[i];
  }
  const hipStream_t s = (hipStream_t)stream;
  return dev_status(timed(AERO_K_GUIDES, s, [&] {
    return launch_guides(p0, v0, a0, d_anchors, d_end_vel, d_end_acc, (double)horizon_T, M, d_coef,
                         s);
  }));
}

int aero_mppi_step(const aero_params* h_prm, const aero_problem* h, int32_t n, void* d_ws,
                   size_t ws_bytes, void* stream) {
  int e = check_params(h_prm);
  if (e) return e;
  e = check_problems(h, n, true);
  if (e) return e;
  MppiPlan pl;
  plan_mppi(h, n, nullptr, h_prm->d_max, pl, kPassAValu, true);
  if (!d_ws || ws_bytes < pl.bytes) return AERO_ERR_WORKSPACE;
  const hipStream_t s = (hipStream_t)stream;
  hipEvent_t* tev = nullptr;
  const int cfg = pick_config(tune_key(h, n), s, &tev);
  plan_mppi(h, n, (char*)d_ws, h_prm->d_max, pl, kPassAConf[cfg].variant, true);
  const DevParams prm = promote(*h_prm);
  // One staged copy for both descriptor arrays (they are adjacent in the workspace).
  const std::vector<char> blob = mppi_blob(pl, n);
  hipError_t he = timed(AERO_K_ROLLOUT, s, [&] {
    return launch_rollout_noise(pl.d_probs, n, pl.total_samples, pl.total_elems, prm, pl.d_sets,
                                pl.total_tiles, blob.data(), blob.size(), s);
  });
  if (he == hipSuccess) he = run_distance(pl, n, cfg, tev, s);
  if (he == hipSuccess && pl.any_nn)
    he = timed(AERO_K_NEAREST, s, [&] { return launch_scatter_nearest(pl.d_sets, n, s); });
  if (he == hipSuccess)
    he = timed(AERO_K_FINALIZE, s, [&] { return launch_finalize(pl.d_probs, n, pl.total_samples, prm, true, s); });
  if (he == hipSuccess)
    he = timed(AERO_K_UPDATE, s, [&] {
      return launch_update(pl.d_probs, n, pl.total_inst, pl.total_rows, prm, s);
    });
  return dev_status(he);
}

int aero_select_best(const aero_params* h_prm, const aero_problem* h, int32_t n, double* d_S2,
                     int32_t* d_best, void* d_ws, size_t ws_bytes, void* stream) {
  int e = check_params(h_prm);
  if (e) return e;
  e = check_problems(h, n, false);
  if (e) return e;
  if (!d_S2 || !d_best) return AERO_ERR_NULL;
  std::vector<DevSelect> sel(n);
  std::vector<QuerySet> sets(n);
  SelectPlan pl;
  pl.sel = sel.data();
  pl.sets = sets.data();
  plan_select(h, n, nullptr, nullptr, nullptr, pl);
  if (!d_ws || ws_bytes < pl.bytes) return AERO_ERR_WORKSPACE;
  plan_select(h, n, (char*)d_ws, d_S2, d_best, pl);
  std::vector<char> blob(select_blob_bytes(pl, n));
  select_blob(pl, n, blob.data());
  return dev_status(run_select(pl, n, promote(*h_prm), blob.data(), blob.size(), true,
                               (hipStream_t)stream));
}

int aero_select_best_noalloc(const aero_params* h_prm, const aero_problem* h, int32_t n,
                             double* d_S2, int32_t* d_best, void* stream) {
  int e = check_params(h_prm);
  if (e) return e;
  e = check_problems(h, n, false);
  if (e) return e;
  if (!d_S2 || !d_best) return AERO_ERR_NULL;
  if (n > AERO_NOALLOC_BATCH_MAX) return AERO_ERR_SHAPE;
  DevSelect sel[AERO_NOALLOC_BATCH_MAX];
  QuerySet sets[AERO_NOALLOC_BATCH_MAX];
  SelectPlan pl;
  pl.sel = sel;
  pl.sets = sets;
  plan_select(h, n, nullptr, nullptr, nullptr, pl);
  if (pl.bytes > (size_t)AERO_NOALLOC_SCRATCH_BYTES) return AERO_ERR_WORKSPACE;
  void* ws = scratch_address();
  if (!ws) return AERO_ERR_DEVICE;
  plan_select(h, n, (char*)ws, d_S2, d_best, pl);
  alignas(16) char blob[kNoAllocBlobBytes];
  const size_t nb = select_blob(pl, n, blob);
  return dev_status(run_select(pl, n, promote(*h_prm), blob, nb, false, (hipStream_t)stream));
}

int aero_mppi_step_backward(const aero_params* h_prm, const aero_problem* h,
                            const float* d_grad_L, float* d_grad_u_nom, float* d_grad_w,
                            void* d_ws, size_t ws_bytes, void* stream) {
  int e = check_params(h_prm);
  if (e) return e;
  e = check_problems(h, 1, true);
  if (e) return e;
  if (!d_grad_u_nom || !d_grad_w) return AERO_ERR_NULL;
  BackwardPlan bp;
  plan_backward(h, nullptr, h_prm->d_max, bp);
  if (!d_ws || ws_bytes < bp.bytes) return AERO_ERR_WORKSPACE;
  // pass A only filters; the shape's tuned forward configuration serves here too
  const int cfg = settled_config(tune_key(h, 1));
  plan_backward(h, (char*)d_ws, h_prm->d_max, bp, kPassAConf[cfg].variant);
  MppiPlan& pl = bp.fwd;
  const hipStream_t s = (hipStream_t)stream;
  const DevParams prm = promote(*h_prm);
  const aero_problem& q = h[0];
  const int64_t MK = (int64_t)q.M * q.K, MN = (int64_t)q.M * q.N;
  const std::vector<char> blob = mppi_blob(pl, 1);
  hipError_t he = timed(AERO_K_ROLLOUT, s, [&] {
    return launch_rollout_noise(pl.d_probs, 1, pl.total_samples, pl.total_elems, prm, pl.d_sets,
                                pl.total_tiles, blob.data(), blob.size(), s);
  });
  if (he == hipSuccess) he = run_distance(pl, 1, cfg, nullptr, s);
  if (he == hipSuccess && q.n_points > 0)
    he = timed(AERO_K_NEAREST, s, [&] { return launch_scatter_nearest(pl.d_sets, 1, s); });
  if (he == hipSuccess)
    he = timed(AERO_K_FINALIZE, s, [&] { return launch_finalize(pl.d_probs, 1, MK, prm, true, s); });
  if (he == hipSuccess)
    he = timed(AERO_K_ADJOINT, s, [&] {
      return launch_adjoint(pl.d_probs, prm, MK, bp.ckpt, bp.seg, bp.gsamp, s);
    });
  if (he == hipSuccess)
    he = timed(AERO_K_GRAD_REDUCE, s, [&] {
      return launch_grad_reduce(pl.d_probs, prm, MN, bp.gsamp, d_grad_L, d_grad_u_nom,
                                d_grad_w, bp.wpart, s);
    });
  return dev_status(he);
}

int aero_mppi_step_backward_indexed(const aero_params* h_prm, const aero_problem* h,
                                    const float* d_grad_L, float* d_grad_u_nom,
                                    float* d_grad_w, void* d_ws, size_t ws_bytes,
                                    void* stream) {
  int e = check_params(h_prm);
  if (e) return e;
  e = check_problems(h, 1, true);
  if (e) return e;
  if (!d_grad_u_nom || !d_grad_w || !h[0].nearest_idx) return AERO_ERR_NULL;
  BackwardPlan bp;
  plan_backward(h, nullptr, h_prm->d_max, bp);
  if (!d_ws || ws_bytes < bp.bytes) return AERO_ERR_WORKSPACE;
  plan_backward(h, (char*)d_ws, h_prm->d_max, bp);
  MppiPlan& pl = bp.fwd;
  // the stored indices are an input: nothing resets or rewrites them
  DevProblem& dp = pl.probs[0];
  dp.nidx = nullptr;
  dp.nn = nullptr;
  dp.nidx_in = h[0].nearest_idx;
  pl.sets[0].nn = nullptr;
  pl.sets[0].nidx = nullptr;
  const hipStream_t s = (hipStream_t)stream;
  const DevParams prm = promote(*h_prm);
  const aero_problem& q = h[0];
  const int64_t MK = (int64_t)q.M * q.K, MN = (int64_t)q.M * q.N;
  const std::vector<char> blob = mppi_blob(pl, 1);
  hipError_t he = timed(AERO_K_ROLLOUT, s, [&] {
    return launch_rollout_noise(pl.d_probs, 1, pl.total_samples, pl.total_elems, prm, pl.d_sets,
                                0, blob.data(), blob.size(), s);  // no distance pass: no cloud boxes
  });
  if (he == hipSuccess)
    he = timed(AERO_K_FINALIZE, s,
               [&] { return launch_finalize(pl.d_probs, 1, MK, prm, false, s); });
  if (he == hipSuccess)
    he = timed(AERO_K_ADJOINT, s, [&] {
      return launch_adjoint(pl.d_probs, prm, MK, bp.ckpt, bp.seg, bp.gsamp, s);
    });
  if (he == hipSuccess)
    he = timed(AERO_K_GRAD_REDUCE, s, [&] {
      return launch_grad_reduce(pl.d_probs, prm, MN, bp.gsamp, d_grad_L, d_grad_u_nom,
                                d_grad_w, bp.wpart, s);
    });
  return dev_status(he);
}

int aero_shift_controls(const float* d_src, int32_t M_src, int32_t N, const int32_t* d_index,
                        int32_t shift, float* d_dst, int32_t M_dst, void* stream) {
  if (!d_src || !d_index || !d_dst) return AERO_ERR_NULL;
  if (M_src < 1 || M_dst < 1 || N < 1 || shift < 0) return AERO_ERR_SHAPE;
  return dev_status(
      launch_shift_controls(d_src, M_src, N, d_index, shift, d_dst, M_dst, (hipStream_t)stream));
}

int aero_step_candidates(const aero_params* h_prm, const float* d_u, const float* d_g, int32_t N,
                         float s0, float beta, int32_t n_candidates, float* d_out, void* stream) {
  int e = check_params(h_prm);
  if (e) return e;
  if (!d_u || !d_g || !d_out) return AERO_ERR_NULL;
  if (N < 1 || n_candidates < 1 || n_candidates > AERO_M_MAX) return AERO_ERR_SHAPE;
  if (!finite(s0) || !finite(beta) || s0 < 0.f || beta < 0.f) return AERO_ERR_PARAM;
  return dev_status(launch_step_candidates(d_u, d_g, N, s0, beta, n_candidates, promote(*h_prm),
                                           d_out, (hipStream_t)stream));
}

int aero_accumulate_cloud(const float* d_ring, int32_t ring_points, const int32_t* d_frame_start,
                          const int32_t* d_frame_offsets, int32_t n_frames, int32_t n_points,
                          const float* d_poses, const float* d_origin, float* d_out,
                          void* stream) {
  if (!d_frame_start || !d_frame_offsets || !d_poses || !d_origin) return AERO_ERR_NULL;
  if (n_frames < 1 || n_frames > AERO_FRAMES_MAX || n_points < 0 || ring_points < 0)
    return AERO_ERR_SHAPE;
  if (n_points == 0) return AERO_OK;
  if (ring_points == 0) return AERO_ERR_SHAPE;
  if (!d_ring || !d_out) return AERO_ERR_NULL;
  return dev_status(launch_accumulate_cloud(d_ring, ring_points, d_frame_start, d_frame_offsets,
                                            n_frames, n_points, d_poses, d_origin, d_out,
                                            (hipStream_t)stream));
}

int aero_advance_state(const aero_params* h_prm, const float* d_x0, const float* d_u, int32_t M,
                       int32_t N, const int32_t* d_index, float* d_x1, void* stream) {
  int e = check_params(h_prm);
  if (e) return e;
  if (!d_x0 || !d_u || !d_index || !d_x1) return AERO_ERR_NULL;
  if (M < 1 || M > AERO_M_MAX || N < 1) return AERO_ERR_SHAPE;
  return dev_status(
      launch_advance_state(d_x0, d_u, M, N, d_index, promote(*h_prm), d_x1, (hipStream_t)stream));
}

int aero_set_pass_a_variant(int variant) {
  if (variant < -1 || variant >= kPassAVariants) return AERO_ERR_PARAM;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_forced_variant = variant;
  return AERO_OK;
}

int aero_read_distance_stats(const aero_problem* h, int32_t n, const void* d_ws,
                             size_t ws_bytes, aero_distance_stats* out) {
  if (!out || !d_ws) return AERO_ERR_NULL;
  const int e = check_problems(h, n, false);
  if (e) return e;
  MppiPlan pl;
  plan_mppi(h, n, nullptr, 1.0f, pl, kPassAValu, true);
  if (ws_bytes < pl.bytes) return AERO_ERR_WORKSPACE;
  plan_mppi(h, n, (char*)const_cast<void*>(d_ws), 1.0f, pl, kPassAValu, true);
  *out = aero_distance_stats{};
  if (pl.item_cap == 0) return AERO_OK;
  // the descriptors as the call wrote them (block sizes of the variant that ran)
  std::vector<QuerySet> sets(n);
  int32_t cnt = 0;
  if (hipMemcpy(sets.data(), pl.d_sets, n * sizeof(QuerySet), hipMemcpyDeviceToHost) !=
          hipSuccess ||
      hipMemcpy(&cnt, pl.item_count, sizeof cnt, hipMemcpyDeviceToHost) != hipSuccess)
    return AERO_ERR_DEVICE;
  const int64_t ni = std::min<int64_t>(std::max(cnt, 0), pl.item_cap);
  std::vector<int2> items(ni);
  std::vector<unsigned char> hit(ni);
  if (ni > 0 && (hipMemcpy(items.data(), pl.items, ni * sizeof(int2), hipMemcpyDeviceToHost) !=
                     hipSuccess ||
                 hipMemcpy(hit.data(), pl.hitf, ni, hipMemcpyDeviceToHost) != hipSuccess))
    return AERO_ERR_DEVICE;
  const int64_t W = sets[0].qpbA / 32;
  const int64_t with_words = std::min<int64_t>(ni, W > 0 ? pl.mask_words / W : 0);
  std::vector<uint32_t> words(with_words * W);
  if (!words.empty() && hipMemcpy(words.data(), pl.hmask, words.size() * 4,
                                  hipMemcpyDeviceToHost) != hipSuccess)
    return AERO_ERR_DEVICE;
  for (int b = 0; b < n; ++b)
    if (sets[b].items) out->positions += sets[b].Q;
  for (int64_t i = 0; i < ni; ++i) {
    const int64_t gqb = items[i].x;
    int b = 0;
    while (b + 1 < n && sets[b + 1].qb_base <= gqb) ++b;
    const QuerySet& S = sets[b];
    const int64_t qb = gqb - S.qb_base;
    const int64_t sub = (int64_t)((unsigned)items[i].y & 0x7fffffffu);
    const int64_t nq = std::min<int64_t>(S.qpbA, S.Q - qb * S.qpbA);
    const int64_t np = std::min<int64_t>(kSubPts, (int64_t)S.n_points - sub * kSubPts);
    if (nq <= 0 || np <= 0) continue;
    out->items += 1;
    out->pairs_a += nq * np;
    if (!hit[i]) continue;
    out->items_b += 1;
    if (i < with_words) {
      int64_t h = 0;
      for (int64_t j = 0; j < W; ++j) {
        const int64_t lo = 32 * j;
        const uint32_t valid = lo >= nq ? 0u : (nq - lo >= 32 ? 0xffffffffu : (1u << (nq - lo)) - 1u);
        h += __builtin_popcount(words[i * W + j] & valid);
      }
      out->pairs_b += h * np;
    } else {
      out->items_whole += 1;
      out->pairs_b += nq * np;
    }
  }
  unsigned long long ev = 0;
  if (count_pass_b_pairs(pl.d_sets, n, pl.items, pl.item_count, pl.hitf, pl.item_cap, &ev) !=
      hipSuccess)
    return AERO_ERR_DEVICE;
  out->pairs_b_eval = (int64_t)ev;
  unsigned long long ea[2] = {0, 0};
  if (count_pass_a_pairs(pl.d_sets, n, pl.items, pl.item_count, pl.item_cap, ea) != hipSuccess)
    return AERO_ERR_DEVICE;
  out->pairs_a_eval = (int64_t)ea[0];
  out->pairs_a_products = (int64_t)ea[1];
  return AERO_OK;
}

int aero_set_pass_a_cull(int on) {
  if (on != 0 && on != 1) return AERO_ERR_PARAM;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_cull = on;
  return AERO_OK;
}

int aero_pass_a_variant(const aero_problem* h_problems, int32_t n_problems) {
  if (!h_problems || n_problems < 1) return -1;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (g_forced_variant >= 0) return g_forced_variant;
  auto it = g_tune.find(tune_key(h_problems, n_problems));
  return (it == g_tune.end() || it->second.choice < 0) ? -1
                                                        : kPassAConf[it->second.choice].variant;
}

int aero_pass_a_grid(const aero_problem* h_problems, int32_t n_problems) {
  if (!h_problems || n_problems < 1) return -1;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (g_forced_variant >= 0) return kPassAConf[g_forced_variant].grid;
  auto it = g_tune.find(tune_key(h_problems, n_problems));
  return (it == g_tune.end() || it->second.choice < 0) ? -1
                                                        : kPassAConf[it->second.choice].grid;
}

int aero_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(g_tmu);
  g_timing.on = on != 0;
  return AERO_OK;
}

int aero_timing_read(int kernel, double* h_total_ms, int64_t* h_launches, int reset) {
  if (!h_total_ms || !h_launches) return AERO_ERR_NULL;
  if (kernel < 0 || kernel >= AERO_K_COUNT) return AERO_ERR_SHAPE;
  std::lock_guard<std::mutex> lk(g_tmu);
  for (auto& r : g_timing.pending) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
      return AERO_ERR_DEVICE;
    g_timing.ms[r.kernel] += ms;
    g_timing.n[r.kernel] += 1;
    g_timing.pool.push_back(r.a);
    g_timing.pool.push_back(r.b);
  }
  g_timing.pending.clear();
  *h_total_ms = g_timing.ms[kernel];
  *h_launches = g_timing.n[kernel];
  if (reset)
    for (int k = 0; k < AERO_K_COUNT; ++k) {
      g_timing.ms[k] = 0.0;
      g_timing.n[k] = 0;
    }
  return AERO_OK;
}

}  // extern "C"
